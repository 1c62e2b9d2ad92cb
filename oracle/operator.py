"""The finite-difference diffusion operator A (section 2.1), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading of the paper.  The PDE of section 2 has diffusion div(D(x) grad u)
with zero normal flux on the boundary.  The per-axis finite-difference formula
of section 2.1 adds a D-weighted 1D Laplacian *and* a one-sided flux
difference on every axis, so that, with constant D, it equals twice the
Laplacian and it neither is symmetric nor conserves mass for variable D (the
matrix A printed there carries the same entries).  This oracle therefore takes
the conservative flux form that the PDE states:

    (A u)_p = (1/h^2) * sum over the 6 face neighbours q of p of K_pq (u_q - u_p)

with the harmonic face mean K_pq = 2 D_p D_q / (D_p + D_q) (0 when both are 0),
so that no flux enters a D = 0 voxel (air/CSF).  Box faces:

* ``noflux``     (the paper's grad u . n = 0): no term, i.e. zero wall flux;
* ``dirichlet0`` (tests only): a ghost value 0 at distance h, coefficient D_p.

The printed form is kept as ``apply_A_paper_literal`` for documentation only.

Arrays are (nx, ny, nz) in C order (z fastest); grid points sit at (i h, j h,
k h) with 0-based indices, i.e. the paper's x_{ijk} shifted by one.
"""

from __future__ import annotations

import itertools

import numpy as np

BCS = ("noflux", "dirichlet0")


def _sl(ax, s):
    out = [slice(None)] * 3
    out[ax] = s
    return tuple(out)


def face_mean(a, b, kind="harmonic"):
    """Face coefficient between two voxel diffusivities."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if kind == "arithmetic":
        return 0.5 * (a + b)
    a, b = np.broadcast_arrays(a, b)
    s = a + b
    out = np.zeros(s.shape, dtype=np.float64)
    nz = s > 0
    out[nz] = 2.0 * a[nz] * b[nz] / s[nz]
    return out


def face_coefficients(D, kind="harmonic"):
    """K on the interior faces: list over axes of arrays with n_ax - 1 planes.

    ``K[ax][..., i, ...]`` couples voxel i and voxel i+1 along ``ax``.
    """
    D = np.asarray(D, dtype=np.float64)
    return [face_mean(D[_sl(ax, slice(0, -1))], D[_sl(ax, slice(1, None))], kind) for ax in range(3)]


def apply_A(u, D, h, bc="noflux", kind="harmonic"):
    """A u for the conservative flux-form operator."""
    assert bc in BCS
    u = np.asarray(u, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    out = np.zeros_like(u)
    for ax, K in enumerate(face_coefficients(D, kind)):
        lo = _sl(ax, slice(0, -1))
        hi = _sl(ax, slice(1, None))
        flux = K * (u[hi] - u[lo])  # flux from the upper voxel into the lower one
        out[lo] += flux
        out[hi] -= flux
        if bc == "dirichlet0":
            first = _sl(ax, slice(0, 1))
            last = _sl(ax, slice(-1, None))
            out[first] -= D[first] * u[first]
            out[last] -= D[last] * u[last]
    return out / (h * h)


def diag_and_offsum(D, h, bc="noflux", kind="harmonic"):
    """Per voxel: |a_pp| and the sum of |a_qp| over q != p."""
    D = np.asarray(D, dtype=np.float64)
    off = np.zeros_like(D)
    ghost = np.zeros_like(D)
    for ax, K in enumerate(face_coefficients(D, kind)):
        off[_sl(ax, slice(0, -1))] += K
        off[_sl(ax, slice(1, None))] += K
        if bc == "dirichlet0":
            ghost[_sl(ax, slice(0, 1))] += D[_sl(ax, slice(0, 1))]
            ghost[_sl(ax, slice(-1, None))] += D[_sl(ax, slice(-1, None))]
    return (off + ghost) / (h * h), off / (h * h)


def norm1(D, h, bc="noflux", kind="harmonic"):
    """||A||_1 = max over columns of the absolute column sum (A is symmetric)."""
    diag, off = diag_and_offsum(D, h, bc, kind)
    return float(np.max(diag + off))


def dense_A(D, h, bc="noflux", kind="harmonic"):
    """Brute-force assembly of A by a loop over voxels and their neighbours.

    Independent of ``apply_A`` (scalar loops, no slicing); for tiny grids only.
    """
    D = np.asarray(D, dtype=np.float64)
    nx, ny, nz = D.shape
    n = nx * ny * nz
    A = np.zeros((n, n))

    def idx(i, j, k):
        return (i * ny + j) * nz + k

    for i, j, k in itertools.product(range(nx), range(ny), range(nz)):
        p = idx(i, j, k)
        for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            a, b, c = i + di, j + dj, k + dk
            if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz:
                dp, dq = D[i, j, k], D[a, b, c]
                if kind == "arithmetic":
                    K = 0.5 * (dp + dq)
                else:
                    K = 0.0 if dp + dq == 0 else 2 * dp * dq / (dp + dq)
                A[p, idx(a, b, c)] += K / h**2
                A[p, p] -= K / h**2
            elif bc == "dirichlet0":
                A[p, p] -= D[i, j, k] / h**2
    return A


def apply_A_paper_literal(u, D, h):
    """The per-axis formula exactly as printed in section 2.1 (documentation only).

    D_p * (u_{+} - 2 u_p + u_{-}) + D_{+} (u_{+} - u_p) - D_p (u_p - u_{-}),
    per axis, divided by h^2, with out-of-grid neighbours taken equal to u_p
    (zero normal derivative).  With constant D this is 2 D times the Laplacian.
    """
    u = np.asarray(u, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    out = np.zeros_like(u)
    for ax in range(3):
        up = np.concatenate([u[_sl(ax, slice(1, None))], u[_sl(ax, slice(-1, None))]], axis=ax)
        um = np.concatenate([u[_sl(ax, slice(0, 1))], u[_sl(ax, slice(0, -1))]], axis=ax)
        Dp = np.concatenate([D[_sl(ax, slice(1, None))], D[_sl(ax, slice(-1, None))]], axis=ax)
        out += D * (up - 2 * u + um) + Dp * (up - u) - D * (u - um)
    return out / (h * h)


# ---------------------------------------------------------------------------
# Label form and the derivative of A with respect to one class diffusivity.
# ---------------------------------------------------------------------------


def class_field(labels, class_D):
    return np.asarray(class_D, dtype=np.float64)[np.asarray(labels)]


def _dK_dDc(la, lb, class_D, c):
    """d K(D_a, D_b) / d D_c for the harmonic mean, per face (label arrays)."""
    cd = np.asarray(class_D, dtype=np.float64)
    da, db = cd[la], cd[lb]
    s = da + db
    same = (la == lb) & (la == c)
    with np.errstate(divide="ignore", invalid="ignore"):
        d_da = np.where(s > 0, 2 * db * db / (s * s), 0.0)
        d_db = np.where(s > 0, 2 * da * da / (s * s), 0.0)
    out = np.where(la == c, d_da, 0.0) + np.where(lb == c, d_db, 0.0)
    # K(D, D) = D exactly, so the derivative is 1 even when D_c = 0.
    out = np.where(same, 1.0, out)
    return out


def apply_dA(u, labels, class_D, c, h, bc="noflux"):
    """(dA/dD_c) u for the harmonic label-form operator."""
    u = np.asarray(u, dtype=np.float64)
    labels = np.asarray(labels)
    out = np.zeros_like(u)
    for ax in range(3):
        lo = _sl(ax, slice(0, -1))
        hi = _sl(ax, slice(1, None))
        dK = _dK_dDc(labels[lo], labels[hi], class_D, c)
        flux = dK * (u[hi] - u[lo])
        out[lo] += flux
        out[hi] -= flux
        if bc == "dirichlet0":
            for end in (slice(0, 1), slice(-1, None)):
                s = _sl(ax, end)
                out[s] -= (labels[s] == c) * u[s]
    return out / (h * h)


class Operator:
    """A bound to a diffusivity field (dense D, or labels plus a class table)."""

    def __init__(self, h, bc="noflux", D=None, labels=None, class_D=None, kind="harmonic"):
        if (D is None) == (labels is None):
            raise ValueError("give exactly one of D or labels")
        self.h = float(h)
        self.bc = bc
        self.kind = kind
        self.labels = None if labels is None else np.asarray(labels)
        self.class_D = None if class_D is None else tuple(float(x) for x in class_D)
        self.D = np.asarray(D, dtype=np.float64) if D is not None else class_field(labels, class_D)

    def __call__(self, u):
        return apply_A(u, self.D, self.h, self.bc, self.kind)

    def norm1(self):
        return norm1(self.D, self.h, self.bc, self.kind)

    def dense(self):
        return dense_A(self.D, self.h, self.bc, self.kind)

    def dA(self, c):
        if self.labels is None:
            raise ValueError("class derivatives need the label form")
        return lambda y: apply_dA(y, self.labels, self.class_D, c, self.h, self.bc)
