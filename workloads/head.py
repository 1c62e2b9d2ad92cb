"""Seeded synthetic heads and initial tumour densities.

Recipe (all randomness from ``numpy.random.default_rng(seed)``, PCG64):

* ellipsoid brain mask centred at ((N-1)/2)(1,1,1) with semi-axes
  (0.45, 0.38, 0.34) * N voxels;
* a smoothed Gaussian random field: standard-normal noise filtered with
  ``scipy.ndimage.gaussian_filter`` at sigma = max(3 N / 128, 1.5) voxels;
* inside the mask the lowest 10 % of the field becomes CSF (class 0, D = 0),
  the highest 13.5 % white matter (class 1, 15 % of the tissue, as the paper
  reports for its 3D head in section 3.3) and the rest gray matter (class 2);
  outside the mask is class 0;
* the tumour seed is a white voxel drawn by the same generator among the white
  voxels at least 9 voxels (3 blob widths) inside the mask, falling back to the
  white voxel farthest from the mask boundary;
* the initial density is a Gaussian blob ``A exp(-|x - c|^2 / (2 sigma^2))``
  (A = 0.8, sigma = 3 voxels) multiplied by the tissue mask (class != 0), so
  that CSF and outside voxels start, and stay, at zero.

Labels are ``uint8`` arrays of shape (N, N, N) in C order with the last (z)
index fastest: flat index ``(i * Ny + j) * Nz + k``.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy import ndimage

# Class diffusivities of the paper's head (Table 1), mm^2/day: 0 air/CSF,
# 1 white matter, 2 gray matter.
CLASS_D_PAPER = (0.0, 0.13, 0.013)

SEMI_AXES = (0.45, 0.38, 0.34)
CSF_FRACTION = 0.10
WHITE_FRACTION = 0.135
BLOB_AMPLITUDE = 0.8
BLOB_SIGMA = 3.0


@dataclass
class Head:
    labels: np.ndarray  # uint8 (N, N, N)
    mask: np.ndarray  # bool (N, N, N), the ellipsoid
    seed_voxel: tuple  # (i, j, k) of the tumour seed
    u0: np.ndarray  # float64 (N, N, N)

    @property
    def shape(self):
        return self.labels.shape


def gaussian_blob(shape, centre, amplitude=BLOB_AMPLITUDE, sigma=BLOB_SIGMA):
    """Gaussian bump on the voxel lattice (coordinates in voxels)."""
    axes = [np.arange(n, dtype=np.float64) for n in shape]
    r2 = np.zeros(shape, dtype=np.float64)
    for ax, (a, c) in enumerate(zip(axes, centre)):
        sh = [1, 1, 1]
        sh[ax] = -1
        r2 = r2 + ((a - c) ** 2).reshape(sh)
    return amplitude * np.exp(-r2 / (2.0 * sigma * sigma))


def uniform_box(n, n_classes_label=1):
    """All-tissue label volume (every voxel carries ``n_classes_label``)."""
    return np.full((n, n, n), n_classes_label, dtype=np.uint8)


def make_head(n: int, seed: int, amplitude=BLOB_AMPLITUDE, sigma=BLOB_SIGMA) -> Head:
    rng = np.random.default_rng(seed)
    c = (n - 1) / 2.0
    idx = np.arange(n, dtype=np.float64)
    a = [s * n for s in SEMI_AXES]
    q = (
        ((idx - c) / a[0]) ** 2
    ).reshape(-1, 1, 1) + (((idx - c) / a[1]) ** 2).reshape(1, -1, 1) + (
        ((idx - c) / a[2]) ** 2
    ).reshape(1, 1, -1)
    mask = q <= 1.0

    smooth = max(3.0 * n / 128.0, 1.5)
    field = ndimage.gaussian_filter(rng.standard_normal((n, n, n)), smooth)
    inside = field[mask]
    lo = np.quantile(inside, CSF_FRACTION)
    hi = np.quantile(inside, 1.0 - WHITE_FRACTION)
    labels = np.zeros((n, n, n), dtype=np.uint8)
    labels[mask] = 2
    labels[mask & (field > hi)] = 1
    labels[mask & (field < lo)] = 0

    dist = ndimage.distance_transform_edt(mask)
    white = labels == 1
    cand = np.argwhere(white & (dist >= 3.0 * sigma))
    if len(cand) > 0:
        seed_voxel = tuple(int(v) for v in cand[rng.integers(len(cand))])
    else:
        dw = np.where(white, dist, -1.0)
        seed_voxel = tuple(int(v) for v in np.unravel_index(np.argmax(dw), dw.shape))

    u0 = gaussian_blob((n, n, n), seed_voxel, amplitude, sigma) * (labels != 0)
    return Head(labels=labels, mask=mask, seed_voxel=seed_voxel, u0=u0)
