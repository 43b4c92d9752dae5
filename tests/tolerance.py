"""Tolerances for comparing GPU results with the FP64 oracle (test helper).

Convolution (FP32 accumulation of K products per output, any order):
    |y - y64| <= TAU_CONV * (|x| (*) |k|)[n]  element-wise, plus a norm-wise
    ||y - y64||_inf <= TAU_CONV * ||y64||_inf.  TAU_CONV is the 1e-5 relative
    target read against the sum of absolute products, since an element-wise
    relative error is meaningless where y ~ 0.

TTC sums: the GPU forms FP32 products and sums them per lane in plain FP32
register blocks of at most BLOCK terms (16 rows x 8 columns at level 0), adds
the block totals of a band in FP32 (at most BLOCKS of them: 256 / 16 + 1 for
the tallest band the tuning allows), adds the owning lanes of a segment (at
most 63) in a pairwise tree of REDUCE_DEPTH rounded additions, and combines
the segments with TwoSum in the finishing pass.  The error of every sum is therefore bounded by
    |s - s64| <= TAU_SUM * sum|terms|,
TAU_SUM = (BLOCK + BLOCKS + REDUCE_DEPTH + 8) * 2^-24; the 8 covers the
rounding of the products and of G.  The bound on A, B, C follows from first-order perturbation
of the normal equations, dv = -M^-1 (dM v + dr), with every sum moved by its
own bound in the worst direction; TTC and FOE follow from C and (A, B).

Residual: with v = (A, B, C) = -M^-1 r and r = (s6, s7, s8), the residual is
the function resid(s) = s9 - r^T M^-1 r of the sums, whose first-order
sensitivities are d resid / d s9 = 1, d resid / d r_i = 2 v_i and
d resid / d M_ij = v_i v_j (each off-diagonal sum sits in M twice).  The bound
adds every sum's own bound times |sensitivity|, doubled as for (A, B, C), plus
the FP64 rounding of evaluating s9 + v . r (8 ulp of the terms' magnitudes).
"""
from __future__ import annotations

import math

import numpy as np

import oracle as O

TAU_CONV = 1e-5
BLOCK = 16 * 8
BLOCKS = 256 // 16 + 1
REDUCE_DEPTH = 6  # pairwise tree over 64 slots
TAU_SUM = (BLOCK + BLOCKS + REDUCE_DEPTH + 8) * 2.0 ** -24


def abs_sums(P0, P1, level, H0, W0):
    """sum |term| for each of the ten sums (oracle arrays, FP64)."""
    ex, ey, et, g = O.level_terms(P0, P1, level, H0, W0)
    prods = (ex * ex, ex * ey, ey * ey, g * ex, g * ey, g * g, ex * et, ey * et, g * et, et * et)
    return np.array([float(np.abs(p).sum()) for p in prods])


def solution_bounds(sums, abs_s, tau=TAU_SUM, safety=2.0):
    """Worst-case first-order bounds (dA, dB, dC, dttc, dx0, dy0) from per-sum bounds tau * abs_s."""
    s = [float(v) for v in sums]
    M, rhs = O.ttc.normal_matrix(s)
    M = np.array(M)
    r = np.array(rhs)
    v = np.linalg.solve(M, r)
    Minv = np.linalg.inv(M)
    # index of each sum in M (symmetric) and in r
    where = {0: [(0, 0)], 1: [(0, 1), (1, 0)], 2: [(1, 1)], 3: [(0, 2), (2, 0)], 4: [(1, 2), (2, 1)], 5: [(2, 2)]}
    dv = np.zeros(3)
    for q in range(9):
        dM = np.zeros((3, 3))
        dr = np.zeros(3)
        if q in where:
            for (i, j) in where[q]:
                dM[i, j] = 1.0
        else:
            dr[q - 6] = -1.0
        sens = -Minv @ (dM @ v - dr)  # d v / d s_q  (M v = r, r = -[s6, s7, s8])
        dv += np.abs(sens) * tau * abs_s[q]
    dv *= safety
    A, B, C = v
    dttc = dv[2] / (C * C) if C != 0 else math.inf
    dx0 = (dv[0] + abs(A / C) * dv[2]) / abs(C) if C != 0 else math.inf
    dy0 = (dv[1] + abs(B / C) * dv[2]) / abs(C) if C != 0 else math.inf
    return dict(A=dv[0], B=dv[1], C=dv[2], ttc=dttc, x0=dx0, y0=dy0)


def resid_bound(sums, abs_s, tau=TAU_SUM, safety=2.0):
    """First-order worst-case bound on the residual from per-sum bounds tau * abs_s."""
    s = [float(v) for v in sums]
    M, rhs = O.ttc.normal_matrix(s)
    v = np.linalg.solve(np.array(M), np.array(rhs))
    a = np.asarray(abs_s, dtype=np.float64)
    sens = np.array([v[0] * v[0], 2 * abs(v[0] * v[1]), v[1] * v[1], 2 * abs(v[0] * v[2]), 2 * abs(v[1] * v[2]),
                     v[2] * v[2], 2 * abs(v[0]), 2 * abs(v[1]), 2 * abs(v[2]), 1.0])
    first = safety * tau * float(np.sum(np.abs(sens) * a))
    rounding = 8 * 2.0 ** -53 * (abs(s[9]) + abs(v[0] * s[6]) + abs(v[1] * s[7]) + abs(v[2] * s[8]))
    return first + rounding


def conv_bound(x, k, mode):
    """TAU_CONV * (|x| (*) |k|) with the oracle (FP64)."""
    return TAU_CONV * O.conv(np.abs(np.asarray(x, dtype=np.float64)), np.abs(np.asarray(k, dtype=np.float64)), mode)
