"""Exponential Euler step of the semi-discrete Fisher-Kolmogorov system, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.2 of the paper:

* the semi-discrete system is u' = A u + f(u) with the logistic reaction
  f(u) = rho u (1 - u) of the PDE in section 2;
* exponential Euler freezes f at u_n over the step, giving
  u_{n+1} = phi0(tau A) u_n + tau phi1(tau A) f(u_n), rewritten with
  phi0 = tau A phi1 + I as the incremental form
  u_{n+1} = u_n + tau phi1(tau A) (A u_n + f(u_n));
* the action tau phi1(tau A) b is the top block of exp(tau B) applied to a unit
  vector, B = [[A, b], [0, 0]] (the augmented matrix, read with the extra
  nilpotent block of the paper dropped since only phi1 is needed and the
  augmented result read as [tau phi1(tau A) b; 1]);
* exp(tau B) is applied as s factors exp(tau B / s), each replaced by its
  degree-m Taylor polynomial.

Applying one degree-m Taylor factor T_m(hB), h = tau/s, to [x; 1] gives
[x + sum_{j=1..m} h^j (A^j x + A^{j-1} b) / j!; 1].  The oracle evaluates that
in nested form: y_1 = h (A x + b), y_j = (h/j) A y_{j-1}, x <- x + sum_j y_j,
starting from x = 0, s times.  ``phi1_action_multinomial`` evaluates the same
polynomial the way the paper's multinomial expansion suggests (powers of the
augmented matrix times precomputed coefficients) for documentation.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np


def reaction(u, rho):
    """f(u) = rho u (1 - u)."""
    return rho * u * (1.0 - u)


def reaction_prime(u, rho):
    return rho * (1.0 - 2.0 * u)


def phi1_action(apply_A, b, tau, s, m):
    """x ~= tau phi1(tau A) b by the scaled, truncated augmented Taylor series."""
    b = np.asarray(b, dtype=np.float64)
    h = tau / s
    x = np.zeros_like(b)
    for _ in range(s):
        y = h * (apply_A(x) + b)
        acc = x + y
        for j in range(2, m + 1):
            y = (h / j) * apply_A(y)
            acc = acc + y
        x = acc
    return x


def taylor_terms(apply_A, x, b, h, m):
    """The m terms y_1..y_m of one sub-step from state x (for the adjoint)."""
    ys = []
    y = h * (apply_A(x) + b)
    ys.append(y)
    for j in range(2, m + 1):
        y = (h / j) * apply_A(y)
        ys.append(y)
    return ys


def rhs(apply_A, u, rho):
    """b = A u + f(u)."""
    return apply_A(u) + reaction(u, rho)


def step(apply_A, u, rho, tau, s, m):
    """One exponential Euler step, incremental form."""
    b = rhs(apply_A, u, rho)
    return u + phi1_action(apply_A, b, tau, s, m)


def advance(apply_A, u0, rho, tau, s, m, nsteps, callback=None):
    u = np.array(u0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        u = step(apply_A, u, rho, tau, s, m)
        if callback is not None:
            callback(n + 1, u)
    return u


def step_direct(apply_A, u, rho, tau, s, m):
    """phi0(tau A) u + tau phi1(tau A) f(u), both by the same Taylor scheme.

    phi0(tau A) u is the top block of exp(tau B) applied to [u; 0]."""
    h = tau / s
    x = np.array(u, dtype=np.float64, copy=True)
    for _ in range(s):
        y = x
        acc = x.copy()
        for j in range(1, m + 1):
            y = (h / j) * apply_A(y)
            acc = acc + y
        x = acc
    return x + phi1_action(apply_A, reaction(u, rho), tau, s, m)


def taylor_power_coefficients(s, m):
    """Coefficients c_k of (sum_{j<=m} z^j / j!)^s, exactly (Fractions)."""
    base = [Fraction(1, 1)]
    f = Fraction(1, 1)
    for j in range(1, m + 1):
        f = f / j
        base.append(f)
    poly = [Fraction(1, 1)]
    for _ in range(s):
        out = [Fraction(0)] * (len(poly) + m)
        for i, a in enumerate(poly):
            if a == 0:
                continue
            for j, c in enumerate(base):
                out[i + j] += a * c
        poly = out
    return poly


def phi1_action_multinomial(apply_A, b, tau, s, m):
    """Same polynomial as ``phi1_action``, expanded in powers of hB (FP64 only).

    The product of s identical degree-m Taylor factors is a single polynomial
    of degree s*m in hB; its coefficients are those of the s-th power of the
    truncated exponential series (the multinomial expansion).  Applied to the
    augmented unit vector: (hB)^k [0; 1] = [h^k A^{k-1} b; 0] for k >= 1.
    """
    h = tau / s
    c = taylor_power_coefficients(s, m)
    p = np.asarray(b, dtype=np.float64) * h  # h A^0 b
    x = float(c[1]) * p
    for k in range(2, len(c)):
        p = h * apply_A(p)
        x = x + float(c[k]) * p
    return x
