"""Choice of the scaling s and the Taylor degree m, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.2 evaluates exp(tau B) v1 as s factors exp(tau B / s), each truncated
after the degree-m Taylor term, "with proper selection of s and m", deferring
to Al-Mohy and Higham for the choice.  The paper states no rule, so this
oracle fixes one (the same rule is documented for the GPU library, which
implements it independently):

  nu = tau * ||A||_1.  Among integers s >= 1 and 1 <= m <= m_max choose the pair
  that minimises the cost s*m (ties to the smaller s) subject to

   (i)  s * theta^(m+1) / (m+1)! <= tol,   theta = nu / s,
   (ii) theta <= theta_max.

Why (i): A is symmetric negative semidefinite and ||A||_2 <= ||A||_1, so every
eigenvalue z of (tau/s) A lies in [-theta, 0].  The Lagrange remainder of the
degree-m Taylor polynomial of e^z is bounded by |z|^(m+1)/(m+1)! there, and
that of phi1 (after m terms) by |z|^m/(m+1)!; over s sub-steps the bounds add.
Why (ii): the partial sums of the Taylor series of e^{-theta} reach about
e^theta / sqrt(2 pi theta) before cancelling, so theta caps the loss of
relative accuracy to rounding.

Defaults: FP64 tol = 1e-13, theta_max = ln 1024; FP32 tol = 1e-6,
theta_max = ln 64.  The FP32 cap bounds the growth of the partial sums at
e^theta / sqrt(2 pi theta), about 12.5, so rounding stays near 1e-6 relative
even for rough vectors; a smaller cap only adds sub-steps.

A lower limit m_min on the degree: the augmented matrix that also carries
phi2 (both columns of the omega block of section 2.2, with the nilpotent J
block) reaches its phi2 vector only through the term (hB)^2 / 2, so a scheme
that needs phi2 takes m >= 2 (at A = 0 the degree-2 truncation is then exact).
"""

from __future__ import annotations

import math

M_MAX = 60
DEFAULTS = {
    "f64": (1e-13, math.log(1024.0)),
    "f32": (1e-6, math.log(64.0)),
}


def remainder_bound(s: int, m: int, theta: float) -> float:
    """s * theta^(m+1) / (m+1)!, built up term by term."""
    t = float(s)
    for k in range(1, m + 2):
        t = t * (theta / k)
    return t


def choose(nu: float, tol: float, theta_max: float, m_max: int = M_MAX, m_min: int = 1):
    """Return (s, m) for the given nu = tau * ||A||_1, with m >= m_min."""
    if not (nu >= 0.0) or math.isinf(nu):
        raise ValueError("nu must be finite and >= 0")
    if not 1 <= m_min <= m_max:
        raise ValueError("need 1 <= m_min <= m_max")
    if nu == 0.0:
        return 1, m_min
    s = max(1, math.ceil(nu / theta_max))
    # ceil can land one short when nu/theta_max is an integer up to rounding
    while nu / s > theta_max:
        s += 1
    best = None
    while True:
        theta = nu / s
        m_found = None
        for m in range(m_min, m_max + 1):
            if remainder_bound(s, m, theta) <= tol:
                m_found = m
                break
        if m_found is not None:
            cost = s * m_found
            if best is None or cost < best[0]:
                best = (cost, s, m_found)
        # Once s alone exceeds the best cost no larger s can win.
        if best is not None and s >= best[0]:
            break
        s += 1
        if s > 100000:
            raise RuntimeError("no admissible (s, m)")
    return best[1], best[2]


def for_dtype(nu: float, dtype: str = "f64", tol: float | None = None, theta_max: float | None = None,
              m_min: int = 1):
    t0, th0 = DEFAULTS[dtype]
    return choose(nu, t0 if tol is None else tol, th0 if theta_max is None else theta_max, m_min=m_min)
