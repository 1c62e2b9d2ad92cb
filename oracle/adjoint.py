"""Discrete adjoint of the exponential Euler advance, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward map is the one ``integrator.advance`` computes, with the plan
(s, m) frozen:

    b_n     = A u_n + f(u_n),            f(u) = rho u (1 - u)
    x_0     = 0;  for sigma = 1..s:  y_1 = h (A x + b_n),  y_j = (h/j) A y_{j-1},
                                     x <- x + y_1 + ... + y_m
    u_{n+1} = u_n + x_s,                 h = tau / s.

The map b -> x_s is a polynomial P(A) applied to b; A is symmetric, hence so is
P(A).  For the loss L = 0.5 ||u_K - u_target||^2 the adjoint state
lambda_n = dL/du_n obeys

    lambda_K = u_K - u_target
    g        = P(A) lambda_{n+1}           (obtained below as the adjoint of b)
    lambda_n = lambda_{n+1} + A g + f'(u_n) * g,      f'(u) = rho (1 - 2u)
    dL/drho += <g, u_n (1 - u_n)>

and for a class diffusivity D_c, with A_c = dA/dD_c:

    dL/dD_c += <g, A_c u_n>  +  sum over sub-steps and terms of
               h <ybar_1, A_c x_{sigma-1}> + sum_{j>=2} (h/j) <ybar_j, A_c y_{j-1}>

where the term adjoints come from running the Taylor recurrence backwards:
ybar_m = xbar, ybar_j = xbar + (h/(j+1)) A ybar_{j+1}; then
xbar <- xbar + h A ybar_1 and bbar += h ybar_1.

Memory: u is checkpointed every ``ckpt_every`` steps; inside a segment the
states are recomputed and kept; inside a step the sub-step states and the
Taylor terms of one sub-step are recomputed.

scheme="linearised" differentiates the paper's linearised step instead
(section 2.1's splitting; see ``rosenbrock``): the Taylor recurrences apply
J_n = A + diag(d_n), d_n = rho (1 - 2 u_n), in place of A (J_n is symmetric
too), and d_n depends on u_n and rho.  Its adjoint

    dbar = sum over sub-steps of h ybar_1 * x_{sigma-1} + sum_{j>=2} (h/j) ybar_j * y_{j-1}

(pointwise products, the same pairs as the class terms) adds
lambda_n += -2 rho dbar and dL/drho += <dbar, 1 - 2 u_n>.  The right-hand side
b_n = A u_n + f(u_n) is the same for both schemes.
"""

from __future__ import annotations

import numpy as np

from .integrator import reaction, reaction_prime, taylor_terms
from .operator import Operator

SCHEMES = ("exp_euler", "linearised")


def _matrix(op, u, rho, scheme):
    """The matrix the step's Taylor recurrences apply: A, or J_n = A + diag(d_n)."""
    if scheme == "exp_euler":
        return op
    if scheme != "linearised":
        raise ValueError(f"unknown scheme {scheme}")
    d = rho * (1.0 - 2.0 * np.asarray(u, dtype=np.float64))
    return lambda x: op(x) + d * x


def _forward_substates(apply_M, b, h, s, m):
    xs = [np.zeros_like(b)]
    for _ in range(s):
        ys = taylor_terms(apply_M, xs[-1], b, h, m)
        xs.append(xs[-1] + sum(ys))
    return xs


def _step(op, u, rho, tau, s, m, scheme="exp_euler"):
    h = tau / s
    b = op(u) + reaction(u, rho)
    return u + _forward_substates(_matrix(op, u, rho, scheme), b, h, s, m)[-1]


def vjp(op: Operator, u0, rho, tau, s, m, nsteps, lam_T, ckpt_every=10, classes=None, scheme="exp_euler"):
    """Returns (grad_u0, grad_rho, {class: grad_D_c}) for the cotangent lam_T."""
    if classes is None:
        classes = list(range(len(op.class_D))) if op.class_D is not None else []
    dA = {c: op.dA(c) for c in classes}
    h = tau / s

    lin = scheme == "linearised"
    ckpts = {}
    u = np.array(u0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        if n % ckpt_every == 0:
            ckpts[n] = u.copy()
        u = _step(op, u, rho, tau, s, m, scheme)

    lam = np.array(lam_T, dtype=np.float64, copy=True)
    g_rho = 0.0
    g_D = {c: 0.0 for c in classes}
    seg_starts = sorted(ckpts)
    for start in reversed(seg_starts):
        stop = min(start + ckpt_every, nsteps)
        states = [ckpts[start]]
        for n in range(start, stop - 1):
            states.append(_step(op, states[-1], rho, tau, s, m, scheme))
        for n in range(stop - 1, start - 1, -1):
            un = states[n - start]
            M = _matrix(op, un, rho, scheme)
            b = op(un) + reaction(un, rho)
            xs = _forward_substates(M, b, h, s, m)
            xbar = lam.copy()
            bbar = np.zeros_like(b)
            dbar = np.zeros_like(b)
            for sigma in range(s, 0, -1):
                x_prev = xs[sigma - 1]
                ys = taylor_terms(M, x_prev, b, h, m)
                ybar = [None] * (m + 1)
                ybar[m] = xbar.copy()
                for j in range(m - 1, 0, -1):
                    ybar[j] = xbar + (h / (j + 1)) * M(ybar[j + 1])
                for c in classes:
                    acc = h * float(np.vdot(ybar[1], dA[c](x_prev)))
                    for j in range(2, m + 1):
                        acc += (h / j) * float(np.vdot(ybar[j], dA[c](ys[j - 2])))
                    g_D[c] += acc
                if lin:
                    dbar = dbar + h * ybar[1] * x_prev
                    for j in range(2, m + 1):
                        dbar = dbar + (h / j) * ybar[j] * ys[j - 2]
                bbar = bbar + h * ybar[1]
                xbar = xbar + h * M(ybar[1])
            g = bbar
            g_rho += float(np.vdot(g, un * (1.0 - un)))
            for c in classes:
                g_D[c] += float(np.vdot(g, dA[c](un)))
            lam = lam + op(g) + reaction_prime(un, rho) * g
            if lin:
                lam = lam - 2.0 * rho * dbar
                g_rho += float(np.vdot(dbar, 1.0 - 2.0 * un))
    return lam, g_rho, g_D


def loss_and_grad(op: Operator, u0, rho, tau, s, m, nsteps, u_target, ckpt_every=10, classes=None,
                  scheme="exp_euler"):
    u = np.array(u0, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        u = _step(op, u, rho, tau, s, m, scheme)
    r = u - u_target
    loss = 0.5 * float(np.vdot(r, r))
    gu0, grho, gD = vjp(op, u0, rho, tau, s, m, nsteps, r, ckpt_every, classes, scheme)
    return loss, gu0, grho, gD


def loss(op_factory, u0, rho, class_D, tau, s, m, nsteps, u_target, scheme="exp_euler"):
    """Forward loss for finite differences; ``op_factory(class_D)`` builds A."""
    op = op_factory(class_D)
    u = np.array(u0, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        u = _step(op, u, rho, tau, s, m, scheme)
    r = u - u_target
    return 0.5 * float(np.vdot(r, r))


def central_fd(op_factory, u0, rho, class_D, tau, s, m, nsteps, u_target, eps=1e-4, classes=(1, 2), directions=(),
               scheme="exp_euler"):
    """Central differences of the loss with the plan frozen.

    Returns (d/drho, {c: d/dD_c}, [directional derivatives along u0 directions]).
    """
    f = lambda r, cd, u: loss(op_factory, u, r, cd, tau, s, m, nsteps, u_target, scheme)  # noqa: E731
    d_rho = (f(rho + eps, class_D, u0) - f(rho - eps, class_D, u0)) / (2 * eps)
    d_D = {}
    for c in classes:
        cp = list(class_D)
        cm = list(class_D)
        cp[c] += eps
        cm[c] -= eps
        d_D[c] = (f(rho, tuple(cp), u0) - f(rho, tuple(cm), u0)) / (2 * eps)
    d_u = [(f(rho, class_D, u0 + eps * v) - f(rho, class_D, u0 - eps * v)) / (2 * eps) for v in directions]
    return d_rho, d_D, d_u
