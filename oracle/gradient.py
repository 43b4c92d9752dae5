"""Image gradient, its magnitude and its direction.  Test infrastructure only.

Discrete Derivatives section: the partial derivatives E_x, E_y of one image
are taken with a small mask applied at every position (multiply the masked
pixels by the mask entries and add), and the gradient's magnitude and angle
are |E| = sqrt(E_x^2 + E_y^2) and the four-quadrant inverse tangent of
(E_y, E_x), in [-pi, pi].  The Convolutions section names the masks in use:
2x2 Roberts, 2x2 Prewitt, 3x3 Prewitt, 3x3 Sobel.

Readings (the figure that shows the masks is missing from the text):
  * FD2 is the Discrete Derivatives section's own mask, (1/2)[[-1, 1], [-1, 1]]
    for E_x and its transpose for E_y (the same as the 2x2 Prewitt mask).
  * The others take their textbook coefficients, scaled so that the ramp
    E = x has E_x = 1: Prewitt 3x3 rows [-1, 0, 1] / 6, Sobel 3x3 rows
    [-1, 0, 1] weighted 1, 2, 1 and / 8.  Roberts takes the two diagonal
    differences E(i+1, j+1) - E(i, j) and E(i+1, j) - E(i, j+1), each / sqrt(2),
    so its axes are the image axes turned by 45 degrees (as the section says).
  * Masks are applied as written (correlation, no flip), at every position
    where they fit (the valid extent): (H-1) x (W-1) for 2x2 masks, (H-2) x
    (W-2) for 3x3 ones; x = column, y = row (downward).
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

STENCILS = ("fd2", "roberts", "prewitt3", "sobel3")


def masks(stencil: str) -> Tuple[np.ndarray, np.ndarray]:
    """(mask for E_x, mask for E_y) as FP64 arrays indexed [row][column]."""
    if stencil == "fd2":
        mx = 0.5 * np.array([[-1.0, 1.0], [-1.0, 1.0]])
        return mx, mx.T.copy()
    if stencil == "roberts":
        r = 1.0 / math.sqrt(2.0)
        return r * np.array([[-1.0, 0.0], [0.0, 1.0]]), r * np.array([[0.0, -1.0], [1.0, 0.0]])
    if stencil == "prewitt3":
        mx = np.array([[-1.0, 0.0, 1.0]] * 3) / 6.0
        return mx, mx.T.copy()
    if stencil == "sobel3":
        mx = np.array([[-1.0, 0.0, 1.0], [-2.0, 0.0, 2.0], [-1.0, 0.0, 1.0]]) / 8.0
        return mx, mx.T.copy()
    raise ValueError(stencil)


def apply_mask(img: np.ndarray, m: np.ndarray) -> np.ndarray:
    """The mask at every position where it fits: out[i][j] = sum m[a][b] img[i+a][j+b]."""
    x = np.asarray(img, dtype=np.float64)
    kh, kw = m.shape
    H, W = x.shape
    out = np.zeros((H - kh + 1, W - kw + 1))
    for a in range(kh):
        for b in range(kw):
            out += m[a, b] * x[a:a + H - kh + 1, b:b + W - kw + 1]
    return out


def gradient(img: np.ndarray, stencil: str = "fd2") -> Dict[str, np.ndarray]:
    """E_x, E_y, magnitude and direction (FP64) of one image."""
    mx, my = masks(stencil)
    ex = apply_mask(img, mx)
    ey = apply_mask(img, my)
    return {"ex": ex, "ey": ey, "mag": np.sqrt(ex * ex + ey * ey), "dir": np.arctan2(ey, ex)}
