"""Pins of the oracle's phi1 + phi2 action and the second-order exponential
Runge-Kutta step (the augmented matrix of section 2.2 with both columns of
its omega block in use).

References outside the Taylor code:
* scipy's dense expm of the (n + 2) x (n + 2) augmented matrix;
* numpy's eigh with the closed forms of phi1 and phi2;
* Heun's method, which the step reduces to when D = 0;
* the exact logistic solution (order 2);
* the reduction to exponential Euler when f(U) = f(u).
"""

import math

import numpy as np
import pytest
import scipy.linalg

from oracle import exprk2 as ek
from oracle import integrator as it
from oracle import operator as op
from oracle import plan
from oracle import reference as ref
from workloads.configs import random_field, random_labels

CLASS_D = (0.0, 0.13, 0.013)


def phi2_scalar(z):
    """(e^z - 1 - z) / z^2, by its series where cancellation would bite."""
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    small = np.abs(z) < 1e-2
    zs = z[small]
    out[small] = 0.5 + zs / 6 + zs**2 / 24 + zs**3 / 120 + zs**4 / 720
    zl = z[~small]
    out[~small] = (np.expm1(zl) - zl) / zl**2
    return out


def dense_augmented(A, b, d, tau):
    """Top block of expm(tau B) e_{n+2}, B = [[A, omega], [0, J]],
    omega = [d / tau, b], J = [[0, 1], [0, 0]]."""
    n = A.shape[0]
    B = np.zeros((n + 2, n + 2))
    B[:n, :n] = A
    B[:n, n] = np.ravel(d) / tau
    B[:n, n + 1] = np.ravel(b)
    B[n, n + 1] = 1.0
    e = np.zeros(n + 2)
    e[n + 1] = 1.0
    w = scipy.linalg.expm(tau * B) @ e
    return w[:n], w[n:]


def _case(shape=(4, 3, 5), bc="noflux", seed=1):
    A_op = op.Operator(0.9, bc=bc, labels=random_labels(shape, 3, seed=seed), class_D=CLASS_D)
    b = random_field(shape, seed=seed + 1, lo=-1, hi=1)
    d = random_field(shape, seed=seed + 2, lo=-1, hi=1)
    return A_op, b, d


@pytest.mark.parametrize("bc", ["noflux", "dirichlet0"])
@pytest.mark.parametrize("tau", [0.5, 7.3, 33.5])
def test_phi12_vs_dense_expm_and_eigh(bc, tau):
    A_op, b, d = _case(bc=bc)
    A = A_op.dense()
    s, m = plan.for_dtype(tau * A_op.norm1(), "f64")
    x = ek.phi12_action(A_op, b, d, tau, s, m).ravel()
    top, tail = dense_augmented(A, b, d, tau)
    np.testing.assert_allclose(tail, [tau, 1.0], rtol=1e-13)  # eta = (tau, 1) after the step
    lam, Q = np.linalg.eigh(A)
    z = tau * lam
    xq = Q @ (tau * ref.phi1_scalar(z) * (Q.T @ b.ravel())) + Q @ (tau * phi2_scalar(z) * (Q.T @ d.ravel()))
    scale = np.linalg.norm(top)
    assert np.linalg.norm(x - top) / scale < 1e-12
    assert np.linalg.norm(x - xq) / scale < 1e-12


def test_each_vector_alone():
    A_op, b, d = _case(shape=(3, 5, 4), seed=11)
    tau = 7.3
    s, m = plan.for_dtype(tau * A_op.norm1(), "f64")
    # b alone: the phi1 action of the plain step (same polynomial)
    np.testing.assert_allclose(ek.phi12_action(A_op, b, None, tau, s, m), it.phi1_action(A_op, b, tau, s, m),
                               rtol=0, atol=1e-14 * np.abs(b).max() * tau)
    # d alone: tau phi2(tau A) d
    lam, Q = np.linalg.eigh(A_op.dense())
    xq = Q @ (tau * phi2_scalar(tau * lam) * (Q.T @ d.ravel()))
    got = ek.phi12_action(A_op, None, d, tau, s, m).ravel()
    assert np.linalg.norm(got - xq) / np.linalg.norm(xq) < 1e-12


@pytest.mark.parametrize("sm", [(1, 1), (1, 2), (2, 1), (3, 3), (1, 8)])
def test_low_degree_truncations_are_the_taylor_polynomial(sm):
    # with m fixed, the scheme is the s-th power of the degree-m Taylor
    # polynomial of exp(hB): compare with that polynomial built on the dense B
    A_op, b, d = _case(shape=(3, 2, 3), seed=21)
    s, m = sm
    tau = 2.0
    A = A_op.dense()
    n = A.shape[0]
    B = np.zeros((n + 2, n + 2))
    B[:n, :n] = A
    B[:n, n] = d.ravel() / tau
    B[:n, n + 1] = b.ravel()
    B[n, n + 1] = 1.0
    hB = (tau / s) * B
    T = np.eye(n + 2)
    term = np.eye(n + 2)
    for j in range(1, m + 1):
        term = term @ hB / j
        T = T + term
    e = np.zeros(n + 2)
    e[n + 1] = 1.0
    expect = (np.linalg.matrix_power(T, s) @ e)[:n]
    got = ek.phi12_action(A_op, b, d, tau, s, m).ravel()
    np.testing.assert_allclose(got, expect, rtol=1e-13, atol=1e-15)


def test_pure_reaction_is_heun():
    # D = 0: A = 0, phi1 = 1, phi2 = 1/2, so the step is Heun's method
    # u + (tau/2)(f(u) + f(u + tau f(u)))
    shape = (3, 4, 5)
    u = random_field(shape, seed=31)
    rho, tau = 0.025, 7.3
    A_op = op.Operator(1.0, D=np.zeros(shape))
    s, m = plan.for_dtype(0.0, "f64", m_min=ek.M_MIN)
    assert (s, m) == (1, 2)
    got = ek.step(A_op, u, rho, tau, s, m)
    f = lambda v: rho * v * (1 - v)  # noqa: E731
    expect = u + 0.5 * tau * (f(u) + f(u + tau * f(u)))
    np.testing.assert_allclose(got, expect, rtol=1e-15, atol=1e-17)


def test_logistic_second_order_convergence():
    rho, u0, T = 0.025, 0.01, 183.8
    exact = u0 * math.exp(rho * T) / (1 + u0 * (math.exp(rho * T) - 1))
    errs = []
    for K in (25, 50, 100, 200):
        A_op = op.Operator(1.0, D=np.zeros((1, 1, 1)))
        u = ek.advance(A_op, np.full((1, 1, 1), u0), rho, T / K, 1, ek.M_MIN, K)
        errs.append(abs(u.item() - exact))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert 3.6 <= r <= 4.4, ratios


def test_linear_problem_is_exp_euler():
    # rho = 0: f = 0, so d = 0 and the step is the (exact) exponential Euler step
    A_op, b, _ = _case(shape=(5, 4, 6), seed=41)
    u = random_field((5, 4, 6), seed=44)
    s, m = plan.for_dtype(7.3 * A_op.norm1(), "f64", m_min=ek.M_MIN)
    np.testing.assert_allclose(ek.step(A_op, u, 0.0, 7.3, s, m), it.step(A_op, u, 0.0, 7.3, s, m), rtol=0,
                               atol=1e-15)


def test_more_accurate_than_exp_euler_on_a_head():
    # against a fine-step reference (the same method at tau / 16)
    from workloads import make_head

    head = make_head(16, 5)
    A_op = op.Operator(1.0, labels=head.labels, class_D=CLASS_D)
    rho, tau, K = 0.025, 7.3, 12
    s, m = plan.for_dtype(tau * A_op.norm1(), "f64", m_min=ek.M_MIN)
    sf, mf = plan.for_dtype(tau / 16 * A_op.norm1(), "f64", m_min=ek.M_MIN)
    fine = ek.advance(A_op, head.u0, rho, tau / 16, sf, mf, 16 * K)
    e2 = np.linalg.norm(ek.advance(A_op, head.u0, rho, tau, s, m, K) - fine)
    e1 = np.linalg.norm(it.advance(A_op, head.u0, rho, tau, s, m, K) - fine)
    assert e2 < 0.2 * e1, (e1, e2)
