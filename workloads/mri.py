"""A seeded synthetic stand-in for the paper's MRI scan (the scan itself is
not available): a uint8 intensity volume of 29 slices of 565 x 532 pixels,
shaped as a head, with the four materials of section 3.1 drawn inside the
intensity range of each.

Geometry: an ellipsoid head whose outer shell is skull, with air outside.
Inside, the brain splits into white (about 15%) and gray matter by a
smoothed random field, the 3-D tissue shares of section 3.3.
"""

from __future__ import annotations

import numpy as np
from scipy import ndimage

SCAN_SHAPE = (29, 565, 532)
# intensity ranges (inclusive) per material: air, white, gray, skull
RANGES = ((0, 1), (2, 115), (116, 240), (241, 255))


def synthetic_scan(shape=SCAN_SHAPE, seed: int = 2402, white_fraction: float = 0.15) -> np.ndarray:
    rng = np.random.default_rng(seed)
    axes = [np.linspace(-1.0, 1.0, n) for n in shape]
    Z, Y, X = np.meshgrid(*axes, indexing="ij")
    r = np.sqrt((Z / 0.95) ** 2 + (Y / 0.85) ** 2 + (X / 0.75) ** 2)
    material = np.zeros(shape, dtype=np.int64)  # air
    brain = r <= 0.86
    material[(r > 0.86) & (r <= 0.95)] = 3  # skull
    coarse = rng.standard_normal((max(2, shape[0] // 3), max(2, shape[1] // 24), max(2, shape[2] // 24)))
    field = ndimage.zoom(coarse, [n / c for n, c in zip(shape, coarse.shape)], order=1)[: shape[0], : shape[1], : shape[2]]
    cut = np.quantile(field[brain], 1.0 - white_fraction)
    material[brain] = np.where(field[brain] > cut, 1, 2)
    out = np.empty(shape, dtype=np.uint8)
    for c, (lo, hi) in enumerate(RANGES):
        sel = material == c
        out[sel] = rng.integers(lo, hi + 1, size=int(sel.sum()), dtype=np.int64).astype(np.uint8)
    return out
