"""Exact semi-discrete references for the phi1 action and the step, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

These do not use the Taylor scheme; they pin it:

* ``dense_phi1_augmented`` - ``scipy.linalg.expm`` of the (n+1)x(n+1) matrix
  [[tau A, tau b], [0, 0]]; its last column holds tau phi1(tau A) b
  (the augmented-matrix identity of section 2.2, one extra row suffices for a
  single phi function);
* ``dense_phi1_paper_augmented`` - the (n+2)x(n+2) construction written in
  section 2.2 with the 2x2 nilpotent block J and columns omega = [b, 0],
  applied to the unit vector at position n+1;
* ``eigh_phi1`` - Q diag(tau phi1(tau lambda)) Q^T b from ``numpy.linalg.eigh``;
* ``modal_phi1`` - for uniform D on a box, A is a Kronecker sum of 1D
  operators whose eigenvectors are DCT-II (no-flux) or DST-I (zero Dirichlet)
  modes, so tau phi1(tau A) b is a diagonal scaling in that basis
  (``scipy.fft.dctn/dstn`` with orthonormal scaling);
* ``modal_apply_A``, ``modal_expm``, ``modal_step``, ``modal_advance`` - the
  operator, exp(t A), the exponential Euler step with the exact phi1 and its
  repetition in the same basis.

phi1(z) = (e^z - 1)/z is evaluated as expm1(z)/z with phi1(0) = 1 (section
2.2 defines phi1 through A^{-1}(e^{tau A} - I); the series sum_k z^k/(k+1)!
is its continuation to singular A).
"""

from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg


def phi1_scalar(z):
    z = np.asarray(z, dtype=np.float64)
    out = np.ones_like(z)
    nz = z != 0
    out[nz] = np.expm1(z[nz]) / z[nz]
    return out


def dense_phi1_augmented(A, b, tau):
    n = A.shape[0]
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = tau * A
    M[:n, n] = tau * np.ravel(b)
    E = scipy.linalg.expm(M)
    return E[:n, n].copy(), E[n, n]


def dense_phi1_paper_augmented(A, b, tau):
    """Returns (top n entries, the two tail entries) of exp(tau B) v1."""
    n = A.shape[0]
    B = np.zeros((n + 2, n + 2))
    B[:n, :n] = A
    B[:n, n] = np.ravel(b)  # omega = [b, 0]
    B[n, n + 1] = 1.0  # J = [[0, 1], [0, 0]]
    v1 = np.zeros(n + 2)
    v1[n] = 1.0
    w = scipy.linalg.expm(tau * B) @ v1
    return w[:n].copy(), w[n:].copy()


def eigh_phi1(A, b, tau):
    lam, Q = np.linalg.eigh(A)
    return Q @ (tau * phi1_scalar(tau * lam) * (Q.T @ np.ravel(b)))


# ---------------------------------------------------------------------------
# Separable (modal) references for uniform D.
# ---------------------------------------------------------------------------


def eigenvalues_1d(n, h, bc="noflux"):
    """Eigenvalues of the 1D operator (u_{i-1} - 2 u_i + u_{i+1}) / h^2.

    no-flux (DCT-II modes cos(pi k (i + 1/2) / n)):       -(4/h^2) sin^2(pi k / (2 n)), k = 0..n-1
    zero Dirichlet (DST-I modes sin(pi k (i + 1)/(n + 1))): -(4/h^2) sin^2(pi k / (2 (n + 1))), k = 1..n
    """
    k = np.arange(n, dtype=np.float64)
    if bc == "noflux":
        return -(4.0 / h**2) * np.sin(np.pi * k / (2.0 * n)) ** 2
    if bc == "dirichlet0":
        return -(4.0 / h**2) * np.sin(np.pi * (k + 1) / (2.0 * (n + 1))) ** 2
    raise ValueError(bc)


def mode_1d(n, k, bc="noflux"):
    """Orthonormal 1D eigenvector number k (k = 0.. for noflux, 0.. = first sine)."""
    i = np.arange(n, dtype=np.float64)
    if bc == "noflux":
        v = np.cos(np.pi * k * (i + 0.5) / n)
    else:
        v = np.sin(np.pi * (k + 1) * (i + 1) / (n + 1))
    return v / np.linalg.norm(v)


def eigenvalues_3d(shape, D, h, bc="noflux"):
    lx, ly, lz = (eigenvalues_1d(n, h, bc) for n in shape)
    return D * (lx[:, None, None] + ly[None, :, None] + lz[None, None, :])


def _fwd(x, bc):
    if bc == "noflux":
        return scipy.fft.dctn(x, type=2, norm="ortho")
    return scipy.fft.dstn(x, type=1, norm="ortho")


def _inv(x, bc):
    if bc == "noflux":
        return scipy.fft.idctn(x, type=2, norm="ortho")
    return scipy.fft.idstn(x, type=1, norm="ortho")


def modal_apply_A(u, D, h, bc="noflux"):
    lam = eigenvalues_3d(u.shape, D, h, bc)
    return _inv(lam * _fwd(np.asarray(u, dtype=np.float64), bc), bc)


def modal_phi1(b, D, h, tau, bc="noflux"):
    lam = eigenvalues_3d(b.shape, D, h, bc)
    return _inv(tau * phi1_scalar(tau * lam) * _fwd(np.asarray(b, dtype=np.float64), bc), bc)


def modal_expm(u, D, h, t, bc="noflux"):
    lam = eigenvalues_3d(u.shape, D, h, bc)
    return _inv(np.exp(t * lam) * _fwd(np.asarray(u, dtype=np.float64), bc), bc)


def modal_step(u, D, h, rho, tau, bc="noflux"):
    """Exact-in-time phi1 of the exponential Euler step, uniform D."""
    b = modal_apply_A(u, D, h, bc) + rho * u * (1.0 - u)
    return u + modal_phi1(b, D, h, tau, bc)


def modal_advance(u0, D, h, rho, tau, nsteps, bc="noflux"):
    u = np.array(u0, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        u = modal_step(u, D, h, rho, tau, bc)
    return u
