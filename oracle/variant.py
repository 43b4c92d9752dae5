"""Time to contact with the alternative derivative stencils and the pyramid
low-pass filter.  Test infrastructure only.

The Convolutions section contrasts the 2x2 masks, whose estimate sits between
pixels, with the centred 3x3 Prewitt and Sobel masks; the Results subsection
down-samples by block averaging followed by a low-pass filter.  This module
runs the least-squares TTC / FOE estimate of the Formulation subsection
(``oracle.ttc``: normal equations, equilibrated 3x3 solve, multi-scale rule)
on derivatives taken either way.

Readings (the paper gives neither the temporal extension of the 3x3 masks nor
the low-pass filter):
  * stencil "cube": the 2x2x2 first-difference cube, exactly ``oracle.ttc``.
  * stencil "prewitt3" / "sobel3": each 3x3 mask is a smoothing across the
    derivative direction times the centred difference (E(j+1) - E(j-1)) / 2;
    smoothing s = [1, 1, 1] / 3 (Prewitt) or [1, 2, 1] / 4 (Sobel).  Over the
    two frames of a pair, as the cube does:
        E_x = (1/2) (M_x * P_0 + M_x * P_1),  E_y likewise with M_y = M_x^T,
        E_t = (s s^T) * (P_1 - P_0),
    at every pixel (i, j) with 1 <= i <= H_l - 2, 1 <= j <= W_l - 2 (masks
    applied as correlations, x = column, y = row downward).
  * positions: a level-l pixel (i, j) has its centre at x = 2^l (j + 1/2) -
    W_0 / 2, y = 2^l (i + 1/2) - H_0 / 2 in base pixels from the base-image
    centre (the cube's positions are the midpoints of these).  Spatial
    derivatives are per base pixel (divided by 2^l), as for the cube.
  * low-pass "binomial3": after each 2x2 block mean, the separable binomial
    filter [1, 2, 1] / 4 along rows and columns, borders clamped (the nearest
    pixel repeats), so every level keeps its size floor(H_l / 2) x floor(W_l / 2).
    Level 0 is never filtered.  "none": the block mean alone (``oracle.pyramid``).
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

from .gradient import apply_mask
from .pyramid import reduce2
from .ttc import select_level, solve_level

STENCILS = ("cube", "prewitt3", "sobel3")
LOWPASS = ("none", "binomial3")

_SMOOTH = {"prewitt3": np.array([1.0, 1.0, 1.0]) / 3.0, "sobel3": np.array([1.0, 2.0, 1.0]) / 4.0}


def lowpass_binomial3(img: np.ndarray) -> np.ndarray:
    """[1, 2, 1] / 4 along the columns then along the rows, borders clamped."""
    x = np.asarray(img, dtype=np.float64)
    H, W = x.shape
    out = np.empty_like(x)
    for i in range(H):
        for j in range(W):
            acc = 0.0
            for a, wa in ((-1, 0.25), (0, 0.5), (1, 0.25)):
                for b, wb in ((-1, 0.25), (0, 0.5), (1, 0.25)):
                    r = min(max(i + a, 0), H - 1)
                    c = min(max(j + b, 0), W - 1)
                    acc += wa * wb * x[r, c]
            out[i, j] = acc
    return out


def pyramid_variant(P: np.ndarray, levels: int, lowpass: str = "none") -> List[np.ndarray]:
    """[P_0, ..., P_{levels-1}]: P_{l+1} = block mean of P_l, then the low-pass filter."""
    if lowpass not in LOWPASS:
        raise ValueError(lowpass)
    out = [np.asarray(P, dtype=np.float64)]
    for _ in range(1, levels):
        nxt = reduce2(out[-1])
        if lowpass == "binomial3":
            nxt = lowpass_binomial3(nxt)
        out.append(nxt)
    return out


def stencil_masks(stencil: str):
    """(M_x, smoothing s s^T) for a 3x3 stencil, FP64, indexed [row][column]."""
    s = _SMOOTH[stencil]
    d = np.array([-1.0, 0.0, 1.0]) / 2.0
    return np.outer(s, d), np.outer(s, s)


def level_terms_variant(P0: np.ndarray, P1: np.ndarray, level: int, H0: int, W0: int, stencil: str):
    """E_x, E_y (per base pixel), E_t and G at every position of one level (FP64)."""
    if stencil == "cube":
        from .ttc import level_terms

        return level_terms(P0, P1, level, H0, W0)
    mx, sm = stencil_masks(stencil)
    my = mx.T.copy()
    s = float(2 ** level)
    ex = 0.5 * (apply_mask(P0, mx) + apply_mask(P1, mx)) / s
    ey = 0.5 * (apply_mask(P0, my) + apply_mask(P1, my)) / s
    et = apply_mask(np.asarray(P1, dtype=np.float64) - np.asarray(P0, dtype=np.float64), sm)
    Hl, Wl = P0.shape
    x = s * (np.arange(1, Wl - 1, dtype=np.float64) + 0.5) - W0 / 2.0
    y = s * (np.arange(1, Hl - 1, dtype=np.float64) + 0.5) - H0 / 2.0
    g = x[None, :] * ex + y[:, None] * ey
    return ex, ey, et, g


def level_sums_variant(P0, P1, level, H0, W0, stencil):
    """The ten sums (correctly rounded, math.fsum) and the number of positions."""
    ex, ey, et, g = level_terms_variant(P0, P1, level, H0, W0, stencil)
    prods = (ex * ex, ex * ey, ey * ey, g * ex, g * ey, g * g, ex * et, ey * et, g * et, et * et)
    return np.array([math.fsum(p.ravel().tolist()) for p in prods]), int(ex.size)


def abs_sums_variant(P0, P1, level, H0, W0, stencil):
    """sum |term| of each of the ten sums (for error bounds)."""
    ex, ey, et, g = level_terms_variant(P0, P1, level, H0, W0, stencil)
    prods = (ex * ex, ex * ey, ey * ey, g * ex, g * ey, g * g, ex * et, ey * et, g * et, et * et)
    return np.array([float(np.abs(p).sum()) for p in prods])


def min_extent(stencil: str) -> int:
    return 2 if stencil == "cube" else 3


def ttc_pair_variant(prev, nxt, levels: int = 1, stencil: str = "cube", lowpass: str = "none") -> List[Dict]:
    """Per-level results for one frame pair with the given stencil and low-pass."""
    if stencil not in STENCILS:
        raise ValueError(stencil)
    prev, nxt = np.asarray(prev), np.asarray(nxt)
    H0, W0 = prev.shape
    p0 = pyramid_variant(prev, levels, lowpass)
    p1 = pyramid_variant(nxt, levels, lowpass)
    k = min_extent(stencil)
    res = []
    for l in range(levels):
        if p0[l].shape[0] < k or p0[l].shape[1] < k:
            raise ValueError(f"level {l} is smaller than {k}x{k}")
        sums, n = level_sums_variant(p0[l], p1[l], l, H0, W0, stencil)
        r = solve_level(sums)
        r.update(level=l, sums=sums, n=n)
        res.append(r)
    return res


def ttc_pair_variant_pick(prev, nxt, levels, stencil="cube", lowpass="none"):
    """(per-level results, the multi-scale choice by the decreasing-TTC rule)."""
    r = ttc_pair_variant(prev, nxt, levels, stencil, lowpass)
    return r, select_level(r)
