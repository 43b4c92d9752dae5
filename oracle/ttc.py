"""Time to contact and focus of expansion from a frame pair.  Test infrastructure only.

Follows the Time to Contact section, Formulation subsection, step by step:

1. Brightness constancy u E_x + v E_y + E_t = 0 (the optical-flow equation).
2. Perspective projection and its time derivative give u = A + C x,
   v = B + C y, hence the linear constraint A E_x + B E_y + C G + E_t = 0 with
   the radial gradient G = x E_x + y E_y.
3. Least squares: minimise the integral of (A E_x + B E_y + C G + E_t)^2; its
   three derivatives give the 3x3 normal equations

     [ S(ExEx) S(ExEy) S(GEx) ] [A]     [ S(ExEt) ]
     [ S(ExEy) S(EyEy) S(GEy) ] [B] = - [ S(EyEt) ]
     [ S(GEx)  S(GEy)  S(GG)  ] [C]     [ S(GEt)  ]

4. Solve, then FOE and TTC: x0 = -A/C, y0 = -B/C, TTC = 1/C.

Readings taken where the paper is silent or inconsistent:
  * The integral becomes an unweighted sum over every full 2x2x2 derivative
    cube of the level.
  * x, y are the cube centres in base-image pixels, origin at the base-image
    centre, x to the right, y downward.  A cube between level-l pixels (i, j)
    and (i+1, j+1) is centred at x = 2^l (j+1) - W0/2, y = 2^l (i+1) - H0/2.
  * Spatial derivatives are expressed per base pixel (E_x,l / 2^l), so A, B,
    x0, y0 are in base pixels at every level; C and TTC are per frame.
  * The sign convention is the operational one u = A + C x (C > 0 for an
    approaching camera); the paper's intermediate u = -(W/Z)(x - x0) carries
    the opposite sign.
  * The 3x3 system is solved by Gaussian elimination with partial pivoting on
    the equilibrated matrix D M D, D = diag(M_ii^-1/2).  The matrix is declared
    singular when a diagonal entry is not positive or a pivot of the
    equilibrated elimination falls below SING_TOL (scale-free: the equilibrated
    matrix has a unit diagonal).
  * residual = sum (A E_x + B E_y + C G + E_t)^2 = S(EtEt) + A S(ExEt) + B S(EyEt) + C S(GEt)
    at the solution.
  * Multi-scale (Results subsection): start at level 0; move to level l+1 while
    its TTC is lower than level l's.  A TTC that is not finite, not positive, or
    whose system is singular counts as +infinity, so any valid estimate
    improves on an invalid one.  Stop at the first non-decrease.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, List, Sequence

import numpy as np

from .horn import horn
from .pyramid import pyramid

SUM_NAMES = ("ExEx", "ExEy", "EyEy", "GEx", "GEy", "GG", "ExEt", "EyEt", "GEt", "EtEt")

STATUS_OK = 0
STATUS_SINGULAR = 1
STATUS_NEED_PREV = 2
STATUS_NONFINITE = 3

SING_TOL = 1e-6


def cube_coords(level: int, Hl: int, Wl: int, H0: int, W0: int):
    """(x[j], y[i]) of the cube centres of a level, base pixels from the base-image centre."""
    s = float(2 ** level)
    x = s * (np.arange(Wl - 1, dtype=np.float64) + 1.0) - W0 / 2.0
    y = s * (np.arange(Hl - 1, dtype=np.float64) + 1.0) - H0 / 2.0
    return x, y


def level_terms(P0: np.ndarray, P1: np.ndarray, level: int, H0: int, W0: int):
    """E_x, E_y (per base pixel), E_t (per frame) and G for every cube of one level (FP64)."""
    ex, ey, et = horn(P0, P1)
    s = float(2 ** level)
    ex = ex / s
    ey = ey / s
    x, y = cube_coords(level, P0.shape[0], P0.shape[1], H0, W0)
    g = x[None, :] * ex + y[:, None] * ey
    return ex, ey, et, g


def _products(ex, ey, et, g):
    return (ex * ex, ex * ey, ey * ey, g * ex, g * ey, g * g, ex * et, ey * et, g * et, et * et)


def level_sums(P0: np.ndarray, P1: np.ndarray, level: int, H0: int, W0: int):
    """The ten sums of the normal equations for one level, each correctly rounded
    (FP64 products, math.fsum), and the cube count n."""
    ex, ey, et, g = level_terms(P0, P1, level, H0, W0)
    sums = np.array([math.fsum(p.ravel().tolist()) for p in _products(ex, ey, et, g)])
    return sums, int(ex.size)


def level_sums_exact(P0: np.ndarray, P1: np.ndarray, level: int, H0: int, W0: int):
    """The ten sums in exact rational arithmetic (small inputs only).

    Valid when the FP64 level images and derivatives are exact (u8 frames and
    rendered f16 frames), which holds for every pyramid level used here."""
    ex, ey, et, g = level_terms(P0, P1, level, H0, W0)
    # the derivative arrays and G are exact dyadic rationals, so Fraction(float) is exact
    fx = [Fraction(v) for v in ex.ravel().tolist()]
    fy = [Fraction(v) for v in ey.ravel().tolist()]
    ft = [Fraction(v) for v in et.ravel().tolist()]
    fg = [Fraction(v) for v in g.ravel().tolist()]
    pairs = ((fx, fx), (fx, fy), (fy, fy), (fg, fx), (fg, fy), (fg, fg), (fx, ft), (fy, ft), (fg, ft), (ft, ft))
    return [sum((a * b for a, b in zip(u, v)), Fraction(0)) for u, v in pairs], len(fx)


def solve3(M, r):
    """Solve the 3x3 system M v = r by Gaussian elimination with partial pivoting (FP64).

    Returns (v, pivots), pivots being the absolute pivot values in elimination order."""
    a = [[float(M[i][j]) for j in range(3)] + [float(r[i])] for i in range(3)]
    pivots = []
    for c in range(3):
        p = max(range(c, 3), key=lambda i: abs(a[i][c]))
        a[c], a[p] = a[p], a[c]
        piv = a[c][c]
        pivots.append(abs(piv))
        if piv == 0.0:
            return [math.nan] * 3, pivots
        for i in range(c + 1, 3):
            f = a[i][c] / piv
            for j in range(c, 4):
                a[i][j] -= f * a[c][j]
    v = [0.0, 0.0, 0.0]
    for i in (2, 1, 0):
        acc = a[i][3]
        for j in range(i + 1, 3):
            acc -= a[i][j] * v[j]
        v[i] = acc / a[i][i]
    return v, pivots


def normal_matrix(sums: Sequence[float]):
    s = [float(v) for v in sums]
    M = [[s[0], s[1], s[3]], [s[1], s[2], s[4]], [s[3], s[4], s[5]]]
    rhs = [-s[6], -s[7], -s[8]]
    return M, rhs


def solve_level(sums: Sequence[float]) -> Dict[str, float]:
    """(A, B, C), TTC, FOE, residual and status from the ten sums of one level."""
    nan = math.nan
    out = dict(A=nan, B=nan, C=nan, ttc=nan, x0=nan, y0=nan, resid=nan, status=STATUS_OK)
    s = [float(v) for v in sums]
    if not all(math.isfinite(v) for v in s):
        out["status"] = STATUS_NONFINITE
        return out
    M, rhs = normal_matrix(s)
    diag = [M[0][0], M[1][1], M[2][2]]
    if min(diag) <= 0.0:
        out["status"] = STATUS_SINGULAR
        return out
    d = [1.0 / math.sqrt(v) for v in diag]
    Me = [[d[i] * M[i][j] * d[j] for j in range(3)] for i in range(3)]
    re = [d[i] * rhs[i] for i in range(3)]
    y, pivots = solve3(Me, re)
    if min(pivots) < SING_TOL:
        out["status"] = STATUS_SINGULAR
        return out
    A, B, C = (d[0] * y[0], d[1] * y[1], d[2] * y[2])
    out.update(A=A, B=B, C=C)
    if C == 0.0:
        out["ttc"] = math.copysign(math.inf, C)
    else:
        out["ttc"] = 1.0 / C
        out["x0"] = -A / C
        out["y0"] = -B / C
    out["resid"] = s[9] + A * s[6] + B * s[7] + C * s[8]
    return out


def ttc_pair(prev: np.ndarray, nxt: np.ndarray, levels: int = 1) -> List[Dict]:
    """Per-level results for one frame pair (levels 0 .. levels-1)."""
    prev = np.asarray(prev)
    nxt = np.asarray(nxt)
    if prev.shape != nxt.shape or prev.ndim != 2:
        raise ValueError("frames must be 2-D and of the same shape")
    H0, W0 = prev.shape
    p0 = pyramid(prev, levels)
    p1 = pyramid(nxt, levels)
    res = []
    for l in range(levels):
        if p0[l].shape[0] < 2 or p0[l].shape[1] < 2:
            raise ValueError(f"level {l} is smaller than 2x2")
        sums, n = level_sums(p0[l], p1[l], l, H0, W0)
        r = solve_level(sums)
        r.update(level=l, sums=sums, n=n)
        res.append(r)
    return res


def _key(r: Dict) -> float:
    t = r["ttc"]
    if r["status"] != STATUS_OK or not math.isfinite(t) or t <= 0.0:
        return math.inf
    return t


def select_level(results: Sequence[Dict]) -> int:
    """Multi-scale choice: descend while the TTC estimate keeps decreasing."""
    l = 0
    while l + 1 < len(results) and _key(results[l + 1]) < _key(results[l]):
        l += 1
    return l


def select_level_residual(results: Sequence[Dict]) -> int:
    """The other reading of the multi-scale rule (Results subsection: "improved"
    read as a better fit): the level whose solution violates the constraint
    least on average, i.e. the smallest residual / number of cubes, among the
    levels with a valid (finite, positive) TTC; the lower level on a tie;
    level 0 when no level is valid."""
    best, best_val = 0, math.inf
    for l, r in enumerate(results):
        if _key(r) == math.inf or r["n"] <= 0:
            continue
        v = r["resid"] / r["n"]
        if v < best_val:
            best, best_val = l, v
    return best


def ttc_sequence(frames, levels: int = 1):
    """[(per-level results, selected level)] for every consecutive pair of a [F, H, W] video."""
    out = []
    for t in range(len(frames) - 1):
        r = ttc_pair(frames[t], frames[t + 1], levels)
        out.append((r, select_level(r)))
    return out
