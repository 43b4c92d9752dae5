"""Direct n-D convolution, FP64 / exact integer.  Test infrastructure only.

Definition (Discrete Derivatives section, the spatial convolution equation, read
with the sum running over the kernel's extent, and as true convolution, i.e.
with the kernel flipped, matching the library ``conv`` routines the paper
benchmarks against in its Benchmarking subsection):

    y[n] = sum_m x[m] * k[n - m],   0 <= n_d <= N_d + K_d - 2   ("full")

The paper applies it to arrays of any rank (Accelerating Convolutions: n-D by
code generation).  Output modes:

    full  : the whole support, extent N + K - 1 per dimension
    same  : full[(K-1)//2 : (K-1)//2 + N]  (extent N, centred)
    valid : the elements that do not touch the zero padding:
            full[min(N,K)-1 : max(N,K)], extent |N - K| + 1; either N >= K in
            every dimension or K >= N in every dimension.
"""
from __future__ import annotations

import itertools
from typing import Iterable, Sequence, Tuple

import numpy as np


def _is_int(a: np.ndarray) -> bool:
    return np.issubdtype(a.dtype, np.integer) or a.dtype == np.bool_


def _work_dtype(x: np.ndarray, k: np.ndarray):
    # Integers accumulate exactly in int64 (|y| <= max|x| * sum|k|, bounded far below 2^63
    # for every input this project produces); everything else in FP64.
    return np.int64 if (_is_int(x) and _is_int(k)) else np.float64


def conv_out_shape(xshape: Sequence[int], kshape: Sequence[int], mode: str) -> Tuple[int, ...]:
    if len(xshape) != len(kshape):
        raise ValueError("x and k must have the same rank")
    if mode == "full":
        return tuple(n + m - 1 for n, m in zip(xshape, kshape))
    if mode == "same":
        return tuple(xshape)
    if mode == "valid":
        ge = all(n >= m for n, m in zip(xshape, kshape))
        le = all(n <= m for n, m in zip(xshape, kshape))
        if not (ge or le):
            raise ValueError("valid mode needs x >= k or k >= x in every dimension")
        return tuple(abs(n - m) + 1 for n, m in zip(xshape, kshape))
    raise ValueError(f"unknown mode {mode!r}")


def _mode_start(xshape, kshape, mode: str) -> Tuple[int, ...]:
    if mode == "full":
        return tuple(0 for _ in xshape)
    if mode == "same":
        return tuple((m - 1) // 2 for m in kshape)
    if mode == "valid":
        return tuple(min(n, m) - 1 for n, m in zip(xshape, kshape))
    raise ValueError(f"unknown mode {mode!r}")


def conv_full(x: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Full-mode convolution by shift-and-add: for every tap t, y[t : t+N] += k[t] * x.

    The taps are visited in row-major order; the arithmetic is FP64 for float
    inputs (every product and sum rounded to FP64) and exact int64 for integers.
    """
    x = np.asarray(x)
    k = np.asarray(k)
    if x.ndim != k.ndim:
        raise ValueError("x and k must have the same rank")
    wd = _work_dtype(x, k)
    xw = x.astype(wd)
    kw = k.astype(wd)
    out_shape = conv_out_shape(x.shape, k.shape, "full")
    y = np.zeros(out_shape, dtype=wd)
    if x.size == 0 or k.size == 0:
        return y
    for t in itertools.product(*(range(m) for m in k.shape)):
        sl = tuple(slice(ti, ti + n) for ti, n in zip(t, x.shape))
        y[sl] += kw[t] * xw
    return y


def conv(x: np.ndarray, k: np.ndarray, mode: str = "full") -> np.ndarray:
    """Convolution in ``mode`` ('full', 'same' or 'valid'), cut out of the full result."""
    x = np.asarray(x)
    k = np.asarray(k)
    shape = conv_out_shape(x.shape, k.shape, mode)
    start = _mode_start(x.shape, k.shape, mode)
    full = conv_full(x, k)
    sl = tuple(slice(s, s + e) for s, e in zip(start, shape))
    return full[sl]


def conv_at(x: np.ndarray, k: np.ndarray, mode: str, index: Iterable[Sequence[int]]) -> np.ndarray:
    """Selected outputs y[n] of ``conv(x, k, mode)``, each summed from the definition.

    y[n] = sum over taps t with 0 <= n_full - t < N of k[t] * x[n_full - t],
    where n_full = n + start(mode).  Used to check outputs of very large
    convolutions one element at a time.  Returns FP64 (int64 for integers).
    """
    x = np.asarray(x)
    k = np.asarray(k)
    wd = _work_dtype(x, k)
    start = _mode_start(x.shape, k.shape, mode)
    out = []
    for n in index:
        nf = [int(a) + s for a, s in zip(n, start)]
        # the taps that land inside x: t in [max(0, nf - N + 1), min(K - 1, nf)]
        lo = [max(0, a - N + 1) for a, N in zip(nf, x.shape)]
        hi = [min(M - 1, a) for a, M in zip(nf, k.shape)]
        if any(h < l for l, h in zip(lo, hi)):
            out.append(wd(0))
            continue
        ksl = tuple(slice(l, h + 1) for l, h in zip(lo, hi))
        xsl = tuple(slice(a - h, a - l + 1) for a, l, h in zip(nf, lo, hi))
        kk = k[ksl].astype(wd)
        xx = x[xsl].astype(wd)
        # x index = nf - t, so the x patch is read in reverse along every axis
        xx = xx[tuple(slice(None, None, -1) for _ in range(xx.ndim))]
        if wd is np.int64:
            out.append(int(np.sum(kk * xx, dtype=np.int64)))
        else:
            out.append(float(np.sum(kk * xx)))
    return np.array(out, dtype=wd)


def conv_bruteforce(x, k, mode: str = "full"):
    """Pure-Python nested loops over output and taps (tiny inputs only); exact for ints."""
    x = np.asarray(x)
    k = np.asarray(k)
    shape = conv_out_shape(x.shape, k.shape, mode)
    start = _mode_start(x.shape, k.shape, mode)
    integer = _is_int(x) and _is_int(k)
    y = np.zeros(shape, dtype=object)
    for n in itertools.product(*(range(e) for e in shape)):
        nf = tuple(a + s for a, s in zip(n, start))
        acc = 0 if integer else 0.0
        for m in itertools.product(*(range(e) for e in x.shape)):
            t = tuple(a - b for a, b in zip(nf, m))
            if all(0 <= ti < K for ti, K in zip(t, k.shape)):
                xv = int(x[m]) if integer else float(x[m])
                kv = int(k[t]) if integer else float(k[t])
                acc += xv * kv
        y[n] = acc
    return y
