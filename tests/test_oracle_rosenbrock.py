"""Pins of the oracle's linearised exponential step (section 2.1's splitting of
the reaction, stepped by section 2.2's phi1 scheme).

References outside the Taylor code and outside ``oracle.rosenbrock``:
* the closed-form scalar map for D = 0;
* scipy's dense expm of the augmented matrix, built on the brute-force A;
* numpy's eigh;
* the exact logistic solution, against which the step converges with order 2;
* the reduction to the plain exponential Euler step when rho = 0;
* brute-force column sums of the dense J_n for the plan bound.
"""

import math

import numpy as np
import pytest

from oracle import integrator as it
from oracle import operator as op
from oracle import plan
from oracle import reference as ref
from oracle import rosenbrock as rb
from workloads import make_head
from workloads.configs import random_field, random_labels

CLASS_D = (0.0, 0.13, 0.013)


def _plan(A_op, rho, tau):
    return plan.for_dtype(tau * rb.norm1_bound(A_op.norm1(), rho), "f64")


def test_reaction_rewriting_identity():
    # section 2.1: F(u_t) = rho (1 - 2 u_{t-1}) u_t + rho u_{t-1}^2 - rho (u_{t-1} - u_t)^2
    rng = np.random.default_rng(3)
    prev, cur, rho = rng.random(50), rng.random(50), 0.025
    lhs = rho * cur * (1 - cur)
    rhs = rho * (1 - 2 * prev) * cur + rho * prev**2 - rho * (prev - cur) ** 2
    np.testing.assert_allclose(lhs, rhs, atol=1e-17)


def test_rhs_equals_plain_rhs():
    # J_n u_n + F_n = A u_n + rho u_n (1 - u_n)
    shape = (6, 5, 7)
    A_op = op.Operator(0.9, labels=random_labels(shape, 3, seed=5), class_D=CLASS_D)
    u = random_field(shape, seed=6)
    a = rb.rhs(A_op, u, 0.03)
    b = it.rhs(A_op, u, 0.03)
    assert np.abs(a - b).max() <= 1e-16 * max(np.abs(b).max(), 1.0) * 8


@pytest.mark.parametrize("tau", [7.3, 60.0])
def test_pure_reaction_closed_form(tau):
    # D = 0: J_n = rho diag(1 - 2 u_n) and each voxel takes the scalar map
    # u + tau phi1(tau rho (1 - 2 u)) rho u (1 - u)
    shape = (3, 4, 5)
    u = random_field(shape, seed=8)
    u.flat[0], u.flat[1], u.flat[2] = 0.0, 1.0, 0.5
    rho = 0.025
    A_op = op.Operator(1.0, D=np.zeros(shape))
    s, m = _plan(A_op, rho, tau)
    got = rb.step(A_op, u, rho, tau, s, m)
    expect = u + tau * ref.phi1_scalar(tau * rho * (1 - 2 * u)) * rho * u * (1 - u)
    np.testing.assert_allclose(got, expect, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("bc", ["noflux", "dirichlet0"])
def test_step_vs_dense_expm(bc):
    shape = (4, 3, 5)
    labels = random_labels(shape, 3, seed=11)
    A_op = op.Operator(0.8, bc=bc, labels=labels, class_D=CLASS_D)
    u = random_field(shape, seed=12)
    rho, tau = 0.05, 7.3
    A = op.dense_A(op.class_field(labels, CLASS_D), 0.8, bc)
    J = A + np.diag(rho * (1 - 2 * u.ravel()))
    b = it.rhs(A_op, u, rho).ravel()
    xe, tail = ref.dense_phi1_augmented(J, b, tau)
    assert tail == pytest.approx(1.0, abs=1e-12)
    xq = ref.eigh_phi1(J, b, tau)
    s, m = _plan(A_op, rho, tau)
    got = rb.step(A_op, u, rho, tau, s, m).ravel() - u.ravel()
    scale = np.linalg.norm(xe)
    assert np.linalg.norm(got - xe) / scale < 1e-12
    assert np.linalg.norm(got - xq) / scale < 1e-12


def test_phi1_action_vs_dense():
    # the standalone action at a given state and vector
    shape = (3, 5, 4)
    A_op = op.Operator(1.0, labels=random_labels(shape, 3, seed=21), class_D=CLASS_D)
    u = random_field(shape, seed=22)
    b = random_field(shape, seed=23, lo=-1, hi=1)
    rho, tau = 0.04, 7.3
    J = A_op.dense() + np.diag(rho * (1 - 2 * u.ravel()))
    s, m = _plan(A_op, rho, tau)
    got = rb.phi1_action(A_op, u, b, rho, tau, s, m).ravel()
    np.testing.assert_allclose(got, ref.eigh_phi1(J, b, tau), atol=1e-13 * np.abs(got).max())


def test_logistic_second_order_convergence():
    # a single voxel with D = 0 is the logistic ODE; the exact Jacobian makes
    # the step second order (the plain step is first order)
    rho, u0, T = 0.025, 0.01, 183.8
    exact = u0 * math.exp(rho * T) / (1 + u0 * (math.exp(rho * T) - 1))
    errs = []
    for K in (25, 50, 100, 200):
        tau = T / K
        A_op = op.Operator(1.0, D=np.zeros((1, 1, 1)))
        s, m = _plan(A_op, rho, tau)
        u = rb.advance(A_op, np.full((1, 1, 1), u0), rho, tau, s, m, K)
        errs.append(abs(u.item() - exact))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert 3.6 <= r <= 4.4, ratios


def test_more_accurate_than_plain_step_at_paper_step():
    # tau = 7.3 d up to the logistic inflection (about half a year from 1%):
    # the plain step is off by about 14%, the linearised step by about 0.3%
    rho, u0, tau, K = 0.025, 0.01, 7.3, 25
    T = tau * K
    exact = u0 * math.exp(rho * T) / (1 + u0 * (math.exp(rho * T) - 1))
    A_op = op.Operator(1.0, D=np.zeros((1, 1, 1)))
    s, m = _plan(A_op, rho, tau)
    u_rb = rb.advance(A_op, np.full((1, 1, 1), u0), rho, tau, s, m, K).item()
    u_ee = it.advance(A_op, np.full((1, 1, 1), u0), rho, tau, s, m, K).item()
    assert abs(u_ee - exact) / exact > 0.1
    assert abs(u_rb - exact) / exact < 0.005


def test_rho_zero_is_plain_step():
    shape = (5, 6, 4)
    A_op = op.Operator(1.0, labels=random_labels(shape, 3, seed=31), class_D=CLASS_D)
    u = random_field(shape, seed=32)
    s, m = _plan(A_op, 0.0, 7.3)
    np.testing.assert_array_equal(rb.step(A_op, u, 0.0, 7.3, s, m), it.step(A_op, u, 0.0, 7.3, s, m))


def test_uniform_state_takes_scalar_map():
    # no-flux and uniform u: A u = 0, so every voxel takes the D = 0 map
    shape = (6, 5, 4)
    A_op = op.Operator(1.0, D=np.full(shape, 0.1))
    rho, tau = 0.025, 7.3
    s, m = _plan(A_op, rho, tau)
    out = rb.advance(A_op, np.full(shape, 0.3), rho, tau, s, m, 3)
    v = 0.3
    for _ in range(3):
        v = v + tau * ref.phi1_scalar(np.array(tau * rho * (1 - 2 * v))).item() * rho * v * (1 - v)
    np.testing.assert_allclose(out, v, rtol=1e-13)


@pytest.mark.parametrize("bc", ["noflux", "dirichlet0"])
def test_norm_bound_and_exact_norm(bc):
    shape = (4, 4, 3)
    A_op = op.Operator(1.0, bc=bc, labels=random_labels(shape, 3, seed=41), class_D=CLASS_D)
    rho = 0.5  # large enough that the diagonal matters
    for seed in range(5):
        u = random_field(shape, seed=50 + seed)
        J = A_op.dense() + np.diag(rho * (1 - 2 * u.ravel()))
        brute = np.abs(J).sum(axis=0).max()
        assert rb.norm1_J(A_op, u, rho) == pytest.approx(brute, rel=1e-14)
        np.testing.assert_allclose(rb.dense_J(A_op, u, rho), J, atol=0)
        assert brute <= rb.norm1_bound(A_op.norm1(), rho) * (1 + 1e-14)
    # attained where D = 0 and the state is 0 or 1
    z = op.Operator(1.0, D=np.zeros(shape))
    uz = np.zeros(shape)
    assert rb.norm1_J(z, uz, rho) == pytest.approx(rb.norm1_bound(0.0, rho))


def test_head_bounds_and_csf():
    head = make_head(20, 9)
    A_op = op.Operator(1.0, labels=head.labels, class_D=CLASS_D)
    s, m = _plan(A_op, 0.025, 7.3)
    u = rb.advance(A_op, head.u0, 0.025, 7.3, s, m, 8)
    assert u.min() >= -1e-12 and u.max() <= 1 + 1e-12
    assert np.all(u[head.labels == 0] == 0.0)
