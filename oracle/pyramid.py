"""2x2 block-average down-sampling.  Test infrastructure only.

Time to Contact, Results: each image is down-sampled by a block averaging
filter; repeating it gives the coarser levels used by the static "Sample k"
methods and by the multi-scale search.  Reading used here: the block is 2x2 and
no further low-pass filter is applied; odd extents are floored (the last row or
column is dropped).

    P_{l+1}[i][j] = 1/4 * sum_{a,b in {0,1}} P_l[2i+a][2j+b],
    H_{l+1} = floor(H_l / 2),  W_{l+1} = floor(W_l / 2)

Computed in FP64, which is exact for u8 frames and for f16 frames whose values
share a common power-of-two grid (the rendered range [16, 240]).
"""
from __future__ import annotations

from typing import List

import numpy as np


def reduce2_loops(P: np.ndarray) -> np.ndarray:
    """One level with explicit loops over the output (small images only)."""
    P = np.asarray(P, dtype=np.float64)
    h, w = P.shape[0] // 2, P.shape[1] // 2
    out = np.empty((h, w), dtype=np.float64)
    for i in range(h):
        for j in range(w):
            out[i, j] = 0.25 * (P[2 * i, 2 * j] + P[2 * i, 2 * j + 1] + P[2 * i + 1, 2 * j] + P[2 * i + 1, 2 * j + 1])
    return out


def reduce2(P: np.ndarray) -> np.ndarray:
    """One level: the mean of every 2x2 block (FP64); the same four-term sum as
    ``reduce2_loops``, in the same order, vectorised."""
    P = np.asarray(P, dtype=np.float64)
    h, w = P.shape[0] // 2, P.shape[1] // 2
    Q = P[: 2 * h, : 2 * w]
    return 0.25 * (Q[0::2, 0::2] + Q[0::2, 1::2] + Q[1::2, 0::2] + Q[1::2, 1::2])


def pyramid(P: np.ndarray, levels: int) -> List[np.ndarray]:
    """[P_0, P_1, ..., P_{levels-1}] with P_0 = P as FP64."""
    if levels < 1:
        raise ValueError("levels must be >= 1")
    out = [np.asarray(P, dtype=np.float64)]
    for _ in range(levels - 1):
        out.append(reduce2(out[-1]))
    return out
