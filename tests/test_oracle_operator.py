"""Pins of the oracle's diffusion operator (section 2.1 read as div(D grad u)).

Each check comes from outside the operator code: a brute-force assembly by
scalar loops, hand-computed two-voxel values, the closed-form eigenpairs of
the 1D Laplacian, conservation and symmetry identities.
"""

import numpy as np
import pytest

from oracle import operator as op
from oracle import reference as ref
from workloads.configs import random_field, random_labels

CLASS_D = (0.0, 0.13, 0.013)


@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 2, 4), (4, 3, 3), (1, 5, 2)])
@pytest.mark.parametrize("bc", ["noflux", "dirichlet0"])
def test_apply_matches_bruteforce(shape, bc):
    labels = random_labels(shape, 3, seed=11)
    D = op.class_field(labels, CLASS_D)
    u = random_field(shape, seed=12, lo=-1, hi=1)
    h = 0.7
    A = op.dense_A(D, h, bc)
    got = op.apply_A(u, D, h, bc)
    np.testing.assert_allclose(got.ravel(), A @ u.ravel(), rtol=0, atol=1e-14)


def test_two_voxel_hand_values():
    # D = 0.13 | 0.013, h = 1: K = 2*0.13*0.013/0.143 = 13/550.
    D = np.array([0.13, 0.013]).reshape(2, 1, 1)
    u = np.array([1.0, 0.0]).reshape(2, 1, 1)
    K = 13.0 / 550.0
    got = op.apply_A(u, D, 1.0).ravel()
    np.testing.assert_allclose(got, [-K, K], rtol=1e-15)
    # ||A||_1: column sum |a_pp| + |a_qp| = 2K
    assert op.norm1(D, 1.0) == pytest.approx(2 * K, rel=1e-15)


def test_zero_diffusivity_blocks_flux():
    # A D = 0 voxel next to tissue: harmonic face mean is 0, nothing leaks in.
    D = np.array([0.13, 0.0, 0.13]).reshape(3, 1, 1)
    u = np.array([1.0, 0.0, 0.0]).reshape(3, 1, 1)
    np.testing.assert_array_equal(op.apply_A(u, D, 1.0).ravel(), [0.0, 0.0, 0.0])


@pytest.mark.parametrize("bc", ["noflux", "dirichlet0"])
def test_eigenpairs_uniform(bc):
    # Separable 1D eigenvectors of the 3-point Laplacian (closed form).
    shape = (6, 5, 7)
    Dc, h = 0.1, 1.3
    D = np.full(shape, Dc)
    for kx, ky, kz in [(0, 0, 0), (1, 0, 2), (5, 4, 6), (2, 3, 1)]:
        vx, vy, vz = (ref.mode_1d(n, k, bc) for n, k in zip(shape, (kx, ky, kz)))
        v = vx[:, None, None] * vy[None, :, None] * vz[None, None, :]
        lam = Dc * sum(ref.eigenvalues_1d(n, h, bc)[k] for n, k in zip(shape, (kx, ky, kz)))
        # the eigenvalue from the sine formula, written out for the first mode
        if bc == "noflux" and (kx, ky, kz) == (1, 0, 2):
            lam_cf = -Dc * 4 / h**2 * (np.sin(np.pi / 12) ** 2 + np.sin(2 * np.pi / 14) ** 2)
            assert lam == pytest.approx(lam_cf, rel=1e-14)
        np.testing.assert_allclose(op.apply_A(v, D, h, bc), lam * v, rtol=0, atol=1e-13)


def test_symmetric_nsd_conservative():
    shape = (4, 3, 5)
    labels = random_labels(shape, 3, seed=3)
    D = op.class_field(labels, CLASS_D)
    A = op.dense_A(D, 1.0)
    np.testing.assert_allclose(A, A.T, atol=0)
    np.testing.assert_allclose(A.sum(axis=0), 0.0, atol=1e-16)
    np.testing.assert_allclose(A.sum(axis=1), 0.0, atol=1e-16)
    assert np.linalg.eigvalsh(A).max() < 1e-15
    # ||A||_1 from the per-voxel sums equals the dense column norm
    assert op.norm1(D, 1.0) == pytest.approx(np.abs(A).sum(axis=0).max(), rel=1e-14)
    Ad = op.dense_A(D, 1.0, "dirichlet0")
    assert op.norm1(D, 1.0, "dirichlet0") == pytest.approx(np.abs(Ad).sum(axis=0).max(), rel=1e-14)


def test_modal_operator_equals_stencil():
    shape = (8, 6, 5)
    u = random_field(shape, seed=5)
    for bc in ("noflux", "dirichlet0"):
        np.testing.assert_allclose(
            ref.modal_apply_A(u, 0.1, 1.0, bc), op.apply_A(u, np.full(shape, 0.1), 1.0, bc), atol=1e-15
        )


def test_paper_literal_form_documented_deviation():
    """The per-axis formula as printed doubles diffusion and leaks mass."""
    shape = (6, 6, 6)
    u = random_field(shape, seed=9)
    Dc = 0.1
    lit = op.apply_A_paper_literal(u, np.full(shape, Dc), 1.0)
    flux = op.apply_A(u, np.full(shape, Dc), 1.0)
    inner = (slice(1, -1),) * 3
    np.testing.assert_allclose(lit[inner], 2 * flux[inner], atol=1e-15)
    labels = random_labels(shape, 3, seed=4)
    D = op.class_field(labels, CLASS_D)
    n = D.size
    cols_lit = np.zeros(n)
    cols_flux = np.zeros(n)
    for q in range(n):
        e = np.zeros(n)
        e[q] = 1.0
        cols_lit[q] = op.apply_A_paper_literal(e.reshape(shape), D, 1.0).sum()
        cols_flux[q] = op.apply_A(e.reshape(shape), D, 1.0).sum()
    assert np.abs(cols_lit).max() > 0.1
    assert np.abs(cols_flux).max() < 1e-15


def test_class_derivative_by_difference():
    shape = (4, 4, 3)
    labels = random_labels(shape, 3, seed=21)
    y = random_field(shape, seed=22)
    cd = (0.02, 0.13, 0.013)
    eps = 1e-6
    for c in range(3):
        cp, cm = list(cd), list(cd)
        cp[c] += eps
        cm[c] -= eps
        fd = (op.apply_A(y, op.class_field(labels, cp), 1.0) - op.apply_A(y, op.class_field(labels, cm), 1.0)) / (
            2 * eps
        )
        np.testing.assert_allclose(op.apply_dA(y, labels, cd, c, 1.0), fd, atol=1e-8)
