"""A second-order exponential Runge-Kutta step, with phi2 from the augmented
matrix, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 1 keeps to the first-order exponential Euler method and notes that
higher-order exponential methods follow the same way.  Section 2.2 builds its
augmented matrix B = [[A, omega], [0, J]] with the 2 x 2 nilpotent block
J = [[0, 1], [0, 0]] and omega an n x 2 block; it fills only one column of
omega, so only phi1 appears.  Filling both columns gives phi2 as well.  For
the augmented state [x; eta], eta in R^2, B maps it to [A x + omega eta;
J eta], and starting from eta = (0, 1) the top block of exp(tau B) [x0; 0, 1]
is

    exp(tau A) x0 + tau phi1(tau A) omega_2 + tau^2 phi2(tau A) omega_1,

with phi1(z) = (e^z - 1)/z and phi2(z) = (e^z - 1 - z)/z^2.  Here omega_2 = b and
omega_1 = d / tau, so the action is tau phi1(tau A) b + tau phi2(tau A) d.

The same scaled Taylor scheme as ``integrator.phi1_action`` evaluates it:
s factors exp(hB), h = tau/s, each truncated after degree m, applied to the
augmented vector.  eta evolves exactly (exp(hJ) eta = eta + h J eta), so after
k sub-steps eta = (k h, 1).

The step (the exponential Runge-Kutta method of order two with one internal
stage at the end of the step):

    U_n     = u_n + tau phi1(tau A) (A u_n + f(u_n))            (the exponential Euler step)
    u_{n+1} = U_n + tau phi2(tau A) (f(U_n) - f(u_n))

One plan (s, m), chosen by the rule of ``plan`` for nu = tau ||A||_1 with the
degree floor m >= 2, serves both actions: the phi2 vector enters the series
only through (hB)^2 / 2, so m = 1 would drop it.  phi2 enters only through
the correction f(U_n) - f(u_n), which is O(tau) against the state.
"""

from __future__ import annotations

import numpy as np

from . import integrator

M_MIN = 2  # the degree floor of the plan (see above)


def phi12_action(apply_A, b, d, tau, s, m):
    """x ~= tau phi1(tau A) b + tau phi2(tau A) d by the scaled, truncated
    Taylor series of the augmented matrix with omega = [d / tau, b].

    b or d may be None (taken as zero)."""
    if b is None and d is None:
        raise ValueError("give b or d")
    ref = b if b is not None else d
    n_shape = np.shape(ref)
    zero = np.zeros(n_shape)
    w2 = zero if b is None else np.asarray(b, dtype=np.float64)  # omega column 2: the phi1 vector
    w1 = zero if d is None else np.asarray(d, dtype=np.float64) / tau  # omega column 1: the phi2 vector
    h = tau / s
    x = np.zeros(n_shape)
    eta = np.array([0.0, 1.0])
    J = np.array([[0.0, 1.0], [0.0, 0.0]])

    def B(v, e):
        return apply_A(v) + e[0] * w1 + e[1] * w2, J @ e

    for _ in range(s):
        acc, acc_eta = x.copy(), eta.copy()
        y, ye = x, eta
        for j in range(1, m + 1):
            by, be = B(y, ye)
            y, ye = (h / j) * by, (h / j) * be
            acc, acc_eta = acc + y, acc_eta + ye
        x, eta = acc, acc_eta
    return x


def step(apply_A, u, rho, tau, s, m):
    """One second-order exponential Runge-Kutta step from u_n."""
    u = np.asarray(u, dtype=np.float64)
    U = u + phi12_action(apply_A, integrator.rhs(apply_A, u, rho), None, tau, s, m)
    d = integrator.reaction(U, rho) - integrator.reaction(u, rho)
    return U + phi12_action(apply_A, None, d, tau, s, m)


def advance(apply_A, u0, rho, tau, s, m, nsteps, callback=None):
    u = np.array(u0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        u = step(apply_A, u, rho, tau, s, m)
        if callback is not None:
            callback(n + 1, u)
    return u
