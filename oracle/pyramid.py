"""FP64 oracle of the Gaussian-pyramid targets of the spatial hierarchy
(Sec. 3.3: the video is fitted coarse to fine against a Gaussian pyramid of
its frames).

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.

Readings (the paper names the pyramid only): level 0 is the frame; level
l + 1 is level l blurred by the separable 5-tap binomial filter
[1, 4, 6, 4, 1] / 16 and decimated by 2 in both directions, keeping the even
rows and columns (output size ceil(H / 2) x ceil(W / 2)); borders are
mirrored without repeating the edge sample (x[-1] = x[1]).
"""
from __future__ import annotations

import numpy as np

KERNEL = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0


def _mirror(i: int, n: int) -> int:
    if n == 1:
        return 0
    while i < 0 or i >= n:
        i = -i if i < 0 else 2 * (n - 1) - i
    return i


def reduce_at(img: np.ndarray, y: int, x: int):
    """Output pixel (y, x) of one REDUCE step on [..., H, W]."""
    img = np.asarray(img, np.float64)
    H, W = img.shape[-2:]
    acc = 0.0
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            acc = acc + KERNEL[dy + 2] * KERNEL[dx + 2] * img[..., _mirror(2 * y + dy, H), _mirror(2 * x + dx, W)]
    return acc


def reduce_level(img: np.ndarray) -> np.ndarray:
    """One REDUCE step on [..., H, W], written out as plain loops over the
    output pixels and the 5 x 5 taps."""
    img = np.asarray(img, np.float64)
    H, W = img.shape[-2:]
    Ho, Wo = (H + 1) // 2, (W + 1) // 2
    out = np.zeros(img.shape[:-2] + (Ho, Wo))
    for y in range(Ho):
        for x in range(Wo):
            out[..., y, x] = reduce_at(img, y, x)
    return out


def pyramid(img: np.ndarray, levels: int):
    """[level 0 = img, level 1, ..., level levels-1]."""
    out = [np.asarray(img, np.float64)]
    for _ in range(levels - 1):
        out.append(reduce_level(out[-1]))
    return out
