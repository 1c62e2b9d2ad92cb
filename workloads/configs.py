"""The standard workloads, as seeded synthetic inputs.

Each function returns plain NumPy inputs (labels, class diffusivities, initial
density, rho, tau, step count).  Sizes can be reduced for tests; the defaults
are the full workloads:

* ``c1_plain``      32^3, uniform D = 0.1, no-flux, Gaussian blob at the centre,
                    tau = 7.3 d, 10 steps (FP64 parity case).
* ``c2_head``       128^3 synthetic head (seed 2402), D = 0.13 / 0.013 / 0,
                    rho = 0.025, tau = 7.3 d, 100 steps (the headline run).
* ``c3_batch``      64 heads, N drawn from {48, 64, 96, 128}, rho ~ U[0.01, 0.05],
                    D_white ~ U[0.05, 0.2], D_gray = D_white / 10, 50 steps.
* ``c4_adjoint``    96^3 head (seed 2404), 50 steps, target from hidden
                    parameters (0.025, 0.13, 0.013) plus N(0, 0.01^2) noise,
                    gradient evaluated at (0.02, 0.10, 0.010).
* ``c5_separable``  256^3, uniform D = 0.1, no-flux, 100 steps.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from .head import CLASS_D_PAPER, gaussian_blob, make_head, uniform_box

TAU = 7.3
RHO = 0.025


@dataclass
class Workload:
    name: str
    labels: np.ndarray  # uint8 (nx, ny, nz), z fastest
    class_D: Tuple[float, ...]
    rho: float
    tau: float
    nsteps: int
    u0: np.ndarray  # float64 (nx, ny, nz)
    h: float = 1.0
    bc: str = "noflux"
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.labels.shape

    @property
    def nvox(self):
        return int(np.prod(self.labels.shape))

    def D(self) -> np.ndarray:
        """Per-voxel diffusivity (float64) from labels and class table."""
        return np.asarray(self.class_D, dtype=np.float64)[self.labels]


def c1_plain(n: int = 32, nsteps: int = 10) -> Workload:
    c = (n - 1) / 2.0
    labels = uniform_box(n, 1)
    u0 = gaussian_blob((n, n, n), (c, c, c))
    return Workload("c1_plain", labels, (0.0, 0.1), RHO, TAU, nsteps, u0)


def c2_head(n: int = 128, nsteps: int = 100, seed: int = 2402) -> Workload:
    head = make_head(n, seed)
    return Workload(
        "c2_head",
        head.labels,
        CLASS_D_PAPER,
        RHO,
        TAU,
        nsteps,
        head.u0,
        extra={"seed_voxel": head.seed_voxel},
    )


@dataclass
class BatchInstance:
    n: int
    rho: float
    class_D: Tuple[float, float, float]
    labels: np.ndarray
    u0: np.ndarray


def c3_batch(count: int = 64, nsteps: int = 50, sizes=(48, 64, 96, 128)) -> Tuple[List[BatchInstance], int]:
    out = []
    for i in range(count):
        seed = 3000 + i
        rng = np.random.default_rng(seed)
        n = int(rng.choice(np.asarray(sizes)))
        rho = float(rng.uniform(0.01, 0.05))
        dw = float(rng.uniform(0.05, 0.2))
        head = make_head(n, seed)
        out.append(BatchInstance(n, rho, (0.0, dw, dw / 10.0), head.labels, head.u0))
    return out, nsteps


def c4_adjoint(n: int = 96, nsteps: int = 50, seed: int = 2404, noise_seed: int = 2405):
    """Calibration workload.

    Returns the workload at the *evaluation* parameters (rho, D_w, D_g) =
    (0.02, 0.10, 0.010), the hidden parameters used to make the target and a
    function that turns a forward result into the noisy target.
    """
    head = make_head(n, seed)
    w = Workload(
        "c4_adjoint",
        head.labels,
        (0.0, 0.10, 0.010),
        0.02,
        TAU,
        nsteps,
        head.u0,
        extra={"hidden": (0.025, 0.13, 0.013), "ckpt_every": 10},
    )
    noise = np.random.default_rng(noise_seed).normal(0.0, 0.01, size=head.labels.shape)
    return w, noise


def c4_synthetic_target(n: int = 96, seed: int = 2404, noise_seed: int = 2405):
    """A target density for gradient parity that does not involve the model:
    a wider Gaussian blob (amplitude 0.9, sigma = 6 voxels) at the tumour seed,
    times the tissue mask, plus N(0, 0.01^2) noise on the tissue."""
    head = make_head(n, seed)
    blob = gaussian_blob(head.labels.shape, head.seed_voxel, amplitude=0.9, sigma=6.0)
    noise = np.random.default_rng(noise_seed).normal(0.0, 0.01, size=head.labels.shape)
    return (blob + noise) * (head.labels != 0)


def c5_separable(n: int = 256, nsteps: int = 100) -> Workload:
    c = (n - 1) / 2.0
    labels = uniform_box(n, 1)
    u0 = gaussian_blob((n, n, n), (c, c, c))
    return Workload("c5_separable", labels, (0.0, 0.1), RHO, TAU, nsteps, u0)


def random_labels(shape, n_classes: int, seed: int) -> np.ndarray:
    """Uniformly random labels, for operator tests on ragged shapes."""
    return np.random.default_rng(seed).integers(0, n_classes, size=shape).astype(np.uint8)


def random_field(shape, seed: int, lo=0.0, hi=1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def make_ragged(shape, seed: int, class_D=CLASS_D_PAPER, rho=RHO, tau=TAU, nsteps=3) -> Workload:
    """Random-label workload on a non-cubic grid (tile tails in every axis)."""
    labels = random_labels(shape, len(class_D), seed)
    u0 = random_field(shape, seed + 1) * (labels != 0)
    return Workload("ragged", labels, tuple(class_D), rho, tau, nsteps, u0)
