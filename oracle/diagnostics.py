"""Label ingestion and tumour diagnostics, plain NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Section 3.1 turns each MRI pixel intensity in [0, 255] into a material by
  fixed thresholds.  The printed ranges are air up to 1, white matter from 1
  to 115, gray matter above 115 up to 240, and skull above 240; they overlap
  at 1.  Reading: each class is bounded above by its threshold and air takes
  the shared value, so label = the number of thresholds strictly below the
  intensity (t = (1, 115, 240): 0 air, 1 white, 2 gray, 3 skull).
* Section 3.5 takes the image values at the points of the finite-difference
  stencil, which is coarser than the scan.  Reading: stencil point i of n
  along an axis of N image samples takes the sample whose cell contains the
  point's cell centre, index floor((2i + 1) N / (2n)), in integer arithmetic.
* Section 3.5 measures the tumour volume as the sum of the density over the
  stencil points divided by their number, after every step.
* Section 3.2 measures the tumour size as the largest distance between two
  grid points holding tumour cells.  Under exponential integration the
  density is positive wherever diffusion reaches, so "holding tumour cells" is
  read as u > threshold, a parameter.  Distances are in grid steps; the size
  in mm is h times that.
"""

from __future__ import annotations

import numpy as np


def sample_index(n: int, N: int) -> np.ndarray:
    """Image index of each of the n stencil points along an axis of N samples."""
    i = np.arange(n, dtype=np.int64)
    return ((2 * i + 1) * N) // (2 * n)


def labels_from_intensity(image, shape, thresholds=(1, 115, 240)):
    """uint8 labels on the stencil grid `shape` from a uint8 image volume."""
    img = np.asarray(image)
    if img.dtype != np.uint8 or img.ndim != 3:
        raise ValueError("image must be a 3-D uint8 array")
    t = [int(v) for v in thresholds]
    if any(b <= a for a, b in zip(t, t[1:])):
        raise ValueError("thresholds must increase")
    ix = [sample_index(n, N) for n, N in zip(shape, img.shape)]
    sampled = img[np.ix_(ix[0], ix[1], ix[2])].astype(np.int64)
    lab = np.zeros(shape, dtype=np.int64)
    for tc in t:
        lab += (sampled > tc)
    return lab.astype(np.uint8)


def tumour_volume(u) -> float:
    """Sum of the density over the grid points, divided by their number."""
    u = np.asarray(u, dtype=np.float64)
    return float(u.sum() / u.size)


def tumour_points(u, threshold):
    """Integer coordinates (M, 3) of the points with u > threshold."""
    return np.argwhere(np.asarray(u) > threshold).astype(np.int64)


def tumour_diameter_sq(u, threshold, block=2048):
    """Largest squared distance (grid steps) between two points with
    u > threshold, by brute force over all pairs; 0 for fewer than two points,
    -1 for none."""
    p = tumour_points(u, threshold)
    if len(p) == 0:
        return -1
    best = 0
    for a in range(0, len(p), block):
        pa = p[a:a + block]
        d = pa[:, None, :] - p[None, :, :]
        best = max(best, int((d * d).sum(axis=2).max()))
    return best


def tumour_diameter_pair(u, threshold, block=2048):
    """(d2, a, b): the largest squared distance and, among the pairs of points
    reaching it, the one with the smallest (a, b), a < b, in linear indices
    (i * ny + j) * nz + k.  (-1, -1, -1) without points, (0, a, a) for one."""
    u = np.asarray(u)
    p = tumour_points(u, threshold)
    if len(p) == 0:
        return -1, -1, -1
    d2 = tumour_diameter_sq(u, threshold, block)
    lin = np.ravel_multi_index(tuple(p.T), u.shape).astype(np.int64)
    if d2 == 0:
        return 0, int(lin[0]), int(lin[0])
    best = None
    for a in range(0, len(p), block):
        d = p[a:a + block, None, :] - p[None, :, :]
        ia, ib = np.nonzero((d * d).sum(axis=2) == d2)
        la, lb = lin[a + ia], lin[ib]
        lo, hi = np.minimum(la, lb), np.maximum(la, lb)
        if len(lo):
            k = np.lexsort((hi, lo))[0]
            cand = (int(lo[k]), int(hi[k]))
            best = cand if best is None else min(best, cand)
    return d2, best[0], best[1]
