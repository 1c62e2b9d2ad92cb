"""The paper's linearised exponential step (exponential Rosenbrock-Euler), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.1, after the matrix A, rewrites the reaction F(u) = rho u (1 - u)
about the previous state: it splits off a part that is linear in the new state,
moves that part into the matrix and keeps the remainder as the source (the
rewritten F and the "new" F that follows it).  Read at the state u_n that the
step starts from:

* the matrix of the step is J_n = A + rho diag(1 - 2 u_n);
* its source is F_n = rho u_n^2.

The paper's superscripts for the previous and the current state coincide when
F is evaluated, so the squared difference of the two states drops out.

The exponential Euler step of section 2.2 applied to u' = J_n u + F_n reads

    u_{n+1} = u_n + tau phi1(tau J_n) (J_n u_n + F_n).

J_n is the Jacobian of A u + f(u) at u_n, which makes this the exponential
Rosenbrock-Euler method, of second order.  Its right-hand side equals the plain
step's, because J_n u_n + F_n = A u_n + rho u_n (1 - u_n).  The phi1 action is
the scaled Taylor scheme of ``integrator.phi1_action`` with J_n in place of A.

Plan.  The rule of ``plan`` needs a bound on tau ||J_n||_1.  Column p of J_n
sums to |a_pp + rho (1 - 2 u_p)| + sum_{q != p} |a_qp|
<= colsum_p(|A|) + rho |1 - 2 u_p|.  So
||J_n||_1 <= ||A||_1 + rho max |1 - 2 u_n| <= ||A||_1 + rho for every state in
[0, 1], the range of the normalised cell density.  One plan, chosen for
nu = tau (||A||_1 + rho), serves every step.  The paper does not say how the
plan follows the state; this reading keeps the plan fixed.
"""

from __future__ import annotations

import numpy as np

from . import integrator
from . import operator as _op


def jacobian_diagonal(u, rho):
    """rho (1 - 2 u_n): what the step adds to the diagonal of A."""
    return rho * (1.0 - 2.0 * np.asarray(u, dtype=np.float64))


def source(u, rho):
    """F_n = rho u_n^2, the source left after the linear part moves into J_n."""
    u = np.asarray(u, dtype=np.float64)
    return rho * u * u


def linearised(apply_A, u, rho):
    """The map x -> J_n x = A x + rho (1 - 2 u_n) x."""
    d = jacobian_diagonal(u, rho)
    return lambda x: apply_A(x) + d * np.asarray(x, dtype=np.float64)


def rhs(apply_A, u, rho):
    """b = J_n u_n + F_n, in the paper's terms."""
    u = np.asarray(u, dtype=np.float64)
    return linearised(apply_A, u, rho)(u) + source(u, rho)


def phi1_action(apply_A, u, b, rho, tau, s, m):
    """x ~= tau phi1(tau J_n) b, J_n taken at the state u."""
    return integrator.phi1_action(linearised(apply_A, u, rho), b, tau, s, m)


def step(apply_A, u, rho, tau, s, m):
    """One linearised exponential step from u_n."""
    u = np.asarray(u, dtype=np.float64)
    return u + phi1_action(apply_A, u, rhs(apply_A, u, rho), rho, tau, s, m)


def advance(apply_A, u0, rho, tau, s, m, nsteps, callback=None):
    u = np.array(u0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        u = step(apply_A, u, rho, tau, s, m)
        if callback is not None:
            callback(n + 1, u)
    return u


def norm1_bound(norm_A1, rho):
    """||A||_1 + rho: a bound on ||J_n||_1 for every state in [0, 1]."""
    return float(norm_A1) + float(rho)


def norm1_J(op, u, rho):
    """||J_n||_1 exactly: max over columns of the absolute column sum."""
    diag_abs, off = _op.diag_and_offsum(op.D, op.h, op.bc, op.kind)
    col = np.abs(-diag_abs + jacobian_diagonal(u, rho)) + off
    return float(np.max(col))


def dense_J(op, u, rho):
    """J_n as a dense matrix (tiny grids): the brute-force A plus the diagonal."""
    return op.dense() + np.diag(np.ravel(jacobian_diagonal(u, rho)))
