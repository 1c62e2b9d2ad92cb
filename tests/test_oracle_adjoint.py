"""Pins of the oracle's discrete adjoint: central finite differences of the
forward loss (plan frozen), the second-order Taylor remainder, and the
symmetry identity adjoint(b) = P(A) lambda; for the plain exponential Euler
step and for the paper's linearised step."""

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import integrator as it
from oracle import operator as op
from oracle import plan
from oracle import rosenbrock as rb
from workloads import make_head
from workloads.configs import random_field


def _setup(n=10, nsteps=4, seed=3):
    head = make_head(n, seed)
    labels = head.labels
    cd = (0.0, 0.10, 0.010)
    A_op = op.Operator(1.0, labels=labels, class_D=cd)
    tau = 7.3
    s, m = plan.for_dtype(tau * A_op.norm1(), "f64")
    rng = np.random.default_rng(seed + 100)
    u0 = head.u0 + 0.05 * rng.random(labels.shape) * (labels != 0)
    target = np.clip(u0 + 0.1 * rng.random(labels.shape), 0, 1) * (labels != 0)
    factory = lambda cdx: op.Operator(1.0, labels=labels, class_D=cdx)  # noqa: E731
    return A_op, factory, u0, target, cd, tau, s, m, nsteps


@pytest.mark.parametrize("scheme", ["exp_euler", "linearised"])
@pytest.mark.parametrize("ckpt", [1, 2, 10])
def test_gradients_vs_central_fd(ckpt, scheme):
    # Central differences at eps = 1e-4 and 5e-5 combined by Richardson
    # extrapolation (error O(eps^4)); the raw differences must also converge
    # at second order towards the adjoint value.
    A_op, factory, u0, target, cd, tau, s, m, K = _setup()
    rho = 0.02
    L, gu0, grho, gD = adj.loss_and_grad(A_op, u0, rho, tau, s, m, K, target, ckpt_every=ckpt, classes=[1, 2],
                                         scheme=scheme)
    rng = np.random.default_rng(7)
    dirs = [rng.standard_normal(u0.shape) for _ in range(2)]
    f1 = adj.central_fd(factory, u0, rho, cd, tau, s, m, K, target, eps=1e-4, directions=dirs, scheme=scheme)
    f2 = adj.central_fd(factory, u0, rho, cd, tau, s, m, K, target, eps=5e-5, directions=dirs, scheme=scheme)

    def check(adjoint_value, a, b):
        rich = (4 * b - a) / 3
        assert adjoint_value == pytest.approx(rich, rel=1e-7)
        if abs(a - adjoint_value) > 1e-9 * abs(adjoint_value):
            assert 3.0 < (a - adjoint_value) / (b - adjoint_value) < 5.0

    check(grho, f1[0], f2[0])
    for c in (1, 2):
        check(gD[c], f1[1][c], f2[1][c])
    for v, a, b in zip(dirs, f1[2], f2[2]):
        check(float(np.vdot(gu0, v)), a, b)


@pytest.mark.parametrize("scheme", ["exp_euler", "linearised"])
def test_taylor_remainder_second_order(scheme):
    A_op, factory, u0, target, cd, tau, s, m, K = _setup(n=8, nsteps=3)
    rho = 0.02
    L0, gu0, _, _ = adj.loss_and_grad(A_op, u0, rho, tau, s, m, K, target, classes=[], scheme=scheme)
    v = np.random.default_rng(1).standard_normal(u0.shape)
    rems = []
    for eps in (1e-1, 5e-2, 2.5e-2):
        Le = adj.loss(factory, u0 + eps * v, rho, cd, tau, s, m, K, target, scheme)
        rems.append(abs(Le - L0 - eps * float(np.vdot(gu0, v))))
    for a, b in zip(rems, rems[1:]):
        assert 3.5 < a / b < 4.5


def test_adjoint_of_b_is_forward_action():
    # For K = 1 and lambda_T = e: grad wrt b is P(A) e = phi1_action(e) since P(A) is symmetric.
    A_op, factory, u0, target, cd, tau, s, m, _ = _setup(n=8)
    e = random_field(u0.shape, seed=3, lo=-1, hi=1)
    # vjp of one step with rho = 0: lambda_0 = e + A P(A) e
    lam0, _, _ = adj.vjp(A_op, u0, 0.0, tau, s, m, 1, e, classes=[])
    expect = e + A_op(it.phi1_action(A_op, e, tau, s, m))
    np.testing.assert_allclose(lam0, expect, atol=1e-14)


def test_forward_matches_integrator():
    # the adjoint's own forward pass is the integrator's step (itself pinned
    # against expm): a mistake there would be consistent with its reverse pass
    A_op, factory, u0, target, cd, tau, s, m, _ = _setup(n=8)
    for rho in (0.0, 0.02):
        np.testing.assert_allclose(adj._step(A_op, u0, rho, tau, s, m), it.step(A_op, u0, rho, tau, s, m),
                                   rtol=0, atol=1e-14)
        np.testing.assert_allclose(adj._step(A_op, u0, rho, tau, s, m, "linearised"),
                                   rb.step(A_op, u0, rho, tau, s, m), rtol=0, atol=1e-14)


def test_linearised_adjoint_at_zero_rho_matches_plain():
    # d_n = 0 when rho = 0: the u0 and class gradients coincide with the plain
    # step's; the rho gradient gains <dbar, 1 - 2u> (the diagonal's derivative)
    A_op, factory, u0, target, cd, tau, s, m, K = _setup(n=8, nsteps=3)
    a = adj.loss_and_grad(A_op, u0, 0.0, tau, s, m, K, target, classes=[1, 2])
    b = adj.loss_and_grad(A_op, u0, 0.0, tau, s, m, K, target, classes=[1, 2], scheme="linearised")
    assert a[0] == pytest.approx(b[0], rel=1e-14)
    np.testing.assert_allclose(a[1], b[1], rtol=0, atol=1e-14 * np.abs(a[1]).max())
    for c in (1, 2):
        assert a[3][c] == pytest.approx(b[3][c], rel=1e-12)
    assert a[2] != pytest.approx(b[2], rel=1e-6)
