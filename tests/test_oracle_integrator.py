"""Pins of the oracle's phi1 action, step and advance (section 2.2).

References outside the Taylor code: scipy's dense expm of the augmented
matrix, numpy's eigh, the DCT/DST modal solution, closed-form eigenmode decay,
the logistic special case D = 0, conservation, symmetry and bounds.
"""

import math

import numpy as np
import pytest

from oracle import integrator as it
from oracle import operator as op
from oracle import plan
from oracle import reference as ref
from workloads import c1_plain, make_head
from workloads.configs import random_field, random_labels

CLASS_D = (0.0, 0.13, 0.013)


def _head_op(n, seed=7):
    head = make_head(n, seed)
    return op.Operator(1.0, labels=head.labels, class_D=CLASS_D), head


@pytest.mark.parametrize("tau", [0.5, 7.3, 33.5])
def test_phi1_action_vs_dense_expm(tau):
    shape = (8, 8, 8)
    labels = random_labels(shape, 3, seed=1)
    A_op = op.Operator(1.0, labels=labels, class_D=CLASS_D)
    b = random_field(shape, seed=2, lo=-1, hi=1)
    A = A_op.dense()
    s, m = plan.for_dtype(tau * A_op.norm1(), "f64")
    x = it.phi1_action(A_op, b, tau, s, m).ravel()
    xe, tail = ref.dense_phi1_augmented(A, b, tau)
    assert tail == pytest.approx(1.0, abs=1e-12)
    xq = ref.eigh_phi1(A, b, tau)
    scale = np.linalg.norm(xe)
    assert np.linalg.norm(x - xe) / scale < 1e-12
    assert np.linalg.norm(x - xq) / scale < 1e-12


def test_paper_augmented_matrix_reading():
    # (n+2) construction with the nilpotent block: top = tau phi1(tau A) b, tail = (1, 0).
    shape = (4, 3, 3)
    labels = random_labels(shape, 3, seed=8)
    A = op.dense_A(op.class_field(labels, CLASS_D), 1.0)
    b = random_field(shape, seed=9).ravel()
    top, tail = ref.dense_phi1_paper_augmented(A, b, 7.3)
    np.testing.assert_allclose(tail, [1.0, 0.0], atol=1e-14)
    np.testing.assert_allclose(top, ref.eigh_phi1(A, b, 7.3), atol=1e-14)


def test_incremental_equals_direct_form():
    A_op, head = _head_op(16)
    u = head.u0
    s, m = plan.for_dtype(7.3 * A_op.norm1(), "f64")
    a = it.step(A_op, u, 0.025, 7.3, s, m)
    b = it.step_direct(A_op, u, 0.025, 7.3, s, m)
    assert np.abs(a - b).max() < 1e-14


def test_multinomial_form_same_polynomial():
    shape = (5, 4, 6)
    labels = random_labels(shape, 3, seed=31)
    A_op = op.Operator(1.0, labels=labels, class_D=CLASS_D)
    b = random_field(shape, seed=32)
    for tau, s, m in [(2.0, 2, 8), (7.3, 3, 10), (7.3, 4, 12)]:
        x1 = it.phi1_action(A_op, b, tau, s, m)
        x2 = it.phi1_action_multinomial(A_op, b, tau, s, m)
        assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-13


def test_taylor_power_coefficients_small():
    # (1 + z + z^2/2)^2 = 1 + 2z + 2z^2 + z^3 + z^4/4
    c = it.taylor_power_coefficients(2, 2)
    assert [float(v) for v in c] == [1.0, 2.0, 2.0, 1.0, 0.25]


@pytest.mark.parametrize("bc", ["noflux", "dirichlet0"])
def test_eigenmode_decay(bc):
    # rho = 0, uniform D: a single mode decays as exp(D lambda t), exactly for the semi-discrete system.
    shape = (12, 10, 8)
    Dc, h, tau, K = 0.1, 1.0, 7.3, 6
    vs = [ref.mode_1d(n, k, bc) for n, k in zip(shape, (2, 1, 3))]
    v = vs[0][:, None, None] * vs[1][None, :, None] * vs[2][None, None, :]
    lam = Dc * sum(ref.eigenvalues_1d(n, h, bc)[k] for n, k in zip(shape, (2, 1, 3)))
    A_op = op.Operator(h, bc=bc, D=np.full(shape, Dc))
    s, m = plan.for_dtype(tau * A_op.norm1(), "f64")
    u = it.advance(A_op, v, 0.0, tau, s, m, K)
    expect = math.exp(lam * tau * K) * v
    assert np.abs(u - expect).max() < 1e-13


def test_logistic_special_case_is_forward_euler():
    # D = 0 everywhere: A = 0, phi1(0) = 1, so the step is u + tau rho u (1 - u) exactly.
    shape = (3, 4, 5)
    u0 = random_field(shape, seed=4)
    A_op = op.Operator(1.0, D=np.zeros(shape))
    assert A_op.norm1() == 0.0
    s, m = plan.for_dtype(0.0, "f64")
    u1 = it.step(A_op, u0, 0.025, 7.3, s, m)
    np.testing.assert_allclose(u1, u0 + 7.3 * 0.025 * u0 * (1 - u0), rtol=1e-15, atol=0)


def test_logistic_first_order_convergence():
    # vs the closed-form logistic solution u0 e^{rt} / (1 + u0 (e^{rt} - 1)).
    rho, u0, T = 0.025, 0.01, 183.8
    exact = u0 * math.exp(rho * T) / (1 + u0 * (math.exp(rho * T) - 1))
    errs = []
    for K in (25, 50, 100, 200):
        tau = T / K
        A_op = op.Operator(1.0, D=np.zeros((1, 1, 1)))
        u = it.advance(A_op, np.full((1, 1, 1), u0), rho, tau, 1, 1, K)
        errs.append(abs(u.item() - exact))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert 1.8 <= r <= 2.2


def test_uniform_state_stays_uniform():
    shape = (6, 5, 4)
    A_op = op.Operator(1.0, D=np.full(shape, 0.1))
    u = np.full(shape, 0.3)
    s, m = plan.for_dtype(7.3 * A_op.norm1(), "f64")
    out = it.advance(A_op, u, 0.025, 7.3, s, m, 3)
    v = 0.3
    for _ in range(3):
        v = v + 7.3 * 0.025 * v * (1 - v)
    np.testing.assert_allclose(out, v, rtol=1e-14)


def test_mass_conservation_no_reaction():
    A_op, head = _head_op(24, seed=17)
    s, m = plan.for_dtype(7.3 * A_op.norm1(), "f64")
    u = it.advance(A_op, head.u0, 0.0, 7.3, s, m, 5)
    assert abs(u.sum() - head.u0.sum()) / head.u0.sum() < 1e-13


def test_bounds_head():
    A_op, head = _head_op(24, seed=19)
    s, m = plan.for_dtype(7.3 * A_op.norm1(), "f64")
    u = it.advance(A_op, head.u0, 0.025, 7.3, s, m, 10)
    assert u.min() >= -1e-12 and u.max() <= 1 + 1e-12
    # CSF/outside voxels never receive tumour cells
    assert np.all(u[head.labels == 0] == 0.0)


def test_reflection_symmetry():
    w = c1_plain(n=12, nsteps=4)
    A_op = op.Operator(1.0, labels=w.labels, class_D=w.class_D)
    s, m = plan.for_dtype(w.tau * A_op.norm1(), "f64")
    u = it.advance(A_op, w.u0, w.rho, w.tau, s, m, w.nsteps)
    for ax in range(3):
        np.testing.assert_allclose(u, np.flip(u, axis=ax), atol=1e-15)


def test_modal_equals_stencil_taylor():
    # Uniform D: the exact modal phi1 and the Taylor scheme agree to the plan tolerance.
    w = c1_plain(n=16, nsteps=3)
    A_op = op.Operator(1.0, D=np.full(w.shape, 0.1))
    s, m = plan.for_dtype(w.tau * A_op.norm1(), "f64")
    u_t = it.advance(A_op, w.u0, w.rho, w.tau, s, m, w.nsteps)
    u_m = ref.modal_advance(w.u0, 0.1, 1.0, w.rho, w.tau, w.nsteps)
    assert np.linalg.norm(u_t - u_m) / np.linalg.norm(u_m) < 1e-12


def test_modal_phi1_vs_dense():
    shape = (5, 4, 6)
    for bc in ("noflux", "dirichlet0"):
        A = op.dense_A(np.full(shape, 0.1), 1.0, bc)
        b = random_field(shape, seed=41)
        np.testing.assert_allclose(
            ref.modal_phi1(b, 0.1, 1.0, 7.3, bc).ravel(), ref.dense_phi1_augmented(A, b, 7.3)[0], atol=1e-13
        )


@pytest.mark.parametrize("bc", ["noflux", "dirichlet0"])
@pytest.mark.parametrize("shape", [(6, 6, 6), (5, 4, 6)])
def test_modal_expm_and_apply_vs_dense(bc, shape):
    # The modal exponential (the reference of the 256^3 pure-diffusion run)
    # against scipy's dense expm of the assembled operator, and the modal A
    # against the assembled matrix itself.
    import scipy.linalg

    A = op.dense_A(np.full(shape, 0.1), 1.0, bc)
    u = random_field(shape, seed=43, lo=-1, hi=1)
    for t in (7.3, 730.0):
        np.testing.assert_allclose(ref.modal_expm(u, 0.1, 1.0, t, bc).ravel(),
                                   scipy.linalg.expm(t * A) @ u.ravel(), atol=1e-13)
    np.testing.assert_allclose(ref.modal_apply_A(u, 0.1, 1.0, bc).ravel(), A @ u.ravel(), atol=1e-14)


def test_modal_step_vs_dense():
    # One exponential Euler step of the modal reference against the same step
    # built from the assembled matrix and scipy's expm of the augmented matrix.
    shape = (6, 5, 4)
    A = op.dense_A(np.full(shape, 0.1), 1.0, "noflux")
    u = random_field(shape, seed=44)
    b = A @ u.ravel() + 0.025 * u.ravel() * (1.0 - u.ravel())
    want = u.ravel() + ref.dense_phi1_augmented(A, b, 7.3)[0]
    np.testing.assert_allclose(ref.modal_step(u, 0.1, 1.0, 0.025, 7.3).ravel(), want, atol=1e-14)


def test_fisher_kpp_front_speed_arithmetic():
    # Section 3.3: 2 sqrt((0.15*0.13 + 0.85*0.013) * 0.025) printed as 0.055 mm/day.
    v = 2 * math.sqrt((0.15 * 0.13 + 0.85 * 0.013) * 0.025)
    assert round(v, 3) == 0.055
