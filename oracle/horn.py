"""First-difference derivative cube E_x, E_y, E_t of a frame pair.  Test infrastructure only.

Discrete Derivatives section: the forward difference E(x+1,y) - E(x,y) from the
limit definition with a one-pixel step, i.e. the two-cell mask [-1, 1] applied
as a sliding weighted sum, and its 2x2 form (1/2)[[-1, 1], [-1, 1]] for E_x
(its transpose for E_y).  The paper gives only the spatial kernel; the reading
used here extends it over the two frames of a pair (the 2x2x2 cube of first
differences), so that the three estimates refer to the same point, the centre
of the cube:

  E_x(i,j) = 1/4 sum_{a,c in {0,1}} [P_c(i+a, j+1) - P_c(i+a, j)]
  E_y(i,j) = 1/4 sum_{b,c in {0,1}} [P_c(i+1, j+b) - P_c(i, j+b)]
  E_t(i,j) = 1/4 sum_{a,b in {0,1}} [P_1(i+a, j+b) - P_0(i+a, j+b)]

for 0 <= i <= H-2, 0 <= j <= W-2 (every full cube, no padding).  x is the
column index j, y the row index i; units are pixels of the level and frames.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def horn(P0: np.ndarray, P1: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(E_x, E_y, E_t), each (H-1) x (W-1), FP64 (exact for u8 / rendered-f16 data)."""
    A = np.asarray(P0, dtype=np.float64)
    B = np.asarray(P1, dtype=np.float64)
    if A.shape != B.shape or A.ndim != 2:
        raise ValueError("frames must be 2-D and of the same shape")
    ex = 0.25 * ((A[:-1, 1:] - A[:-1, :-1]) + (A[1:, 1:] - A[1:, :-1])
                 + (B[:-1, 1:] - B[:-1, :-1]) + (B[1:, 1:] - B[1:, :-1]))
    ey = 0.25 * ((A[1:, :-1] - A[:-1, :-1]) + (A[1:, 1:] - A[:-1, 1:])
                 + (B[1:, :-1] - B[:-1, :-1]) + (B[1:, 1:] - B[:-1, 1:]))
    et = 0.25 * ((B[:-1, :-1] - A[:-1, :-1]) + (B[:-1, 1:] - A[:-1, 1:])
                 + (B[1:, :-1] - A[1:, :-1]) + (B[1:, 1:] - A[1:, 1:]))
    return ex, ey, et


def horn_numerators(P0: np.ndarray, P1: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """4*E_x, 4*E_y, 4*E_t as exact int64 for integer frames (u8 sources)."""
    A = np.asarray(P0).astype(np.int64)
    B = np.asarray(P1).astype(np.int64)
    if A.shape != B.shape or A.ndim != 2:
        raise ValueError("frames must be 2-D and of the same shape")
    nx = (A[:-1, 1:] - A[:-1, :-1]) + (A[1:, 1:] - A[1:, :-1]) + (B[:-1, 1:] - B[:-1, :-1]) + (B[1:, 1:] - B[1:, :-1])
    ny = (A[1:, :-1] - A[:-1, :-1]) + (A[1:, 1:] - A[:-1, 1:]) + (B[1:, :-1] - B[:-1, :-1]) + (B[1:, 1:] - B[:-1, 1:])
    nt = (B[:-1, :-1] - A[:-1, :-1]) + (B[:-1, 1:] - A[:-1, 1:]) + (B[1:, :-1] - A[1:, :-1]) + (B[1:, 1:] - A[1:, 1:])
    return nx, ny, nt
