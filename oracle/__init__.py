"""FP64 CPU oracle for the exponential-Euler Fisher-Kolmogorov step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, tables or helpers); both sides only share the
seeded input generators of ``workloads``.

Plain, slow, obviously-correct NumPy/SciPy in float64:

* ``operator``   the finite-difference diffusion operator A of section 2.1
                 (Eq. for the semi-discrete system, matrix A), read as the
                 conservative flux form of div(D grad u) in the PDE of
                 section 2 with harmonic face means;
* ``plan``       the choice of the scaling s and Taylor degree m (section 2.2
                 only asks for a "proper selection"; the rule is stated there);
* ``integrator`` reaction term, the augmented-matrix scaled Taylor action of
                 tau*phi1(tau*A) (section 2.2), the exponential Euler step in
                 its incremental form u + tau*phi1(tau*A)(A u + f(u)), and the
                 multi-step advance;
* ``reference``  exact semi-discrete references: dense expm of the augmented
                 matrix, eigen-decomposition, and the separable DCT/DST modal
                 solution for uniform D;
* ``rosenbrock`` the paper's linearised step: the linear part of the reaction
                 moved into the matrix, J_n = A + rho diag(1 - 2 u_n), source
                 rho u_n^2 (section 2.1), stepped by the same phi1 scheme
                 (exponential Rosenbrock-Euler);
* ``exprk2``     tau phi1(tau A) b + tau phi2(tau A) d from the augmented matrix
                 with both columns of its omega block (section 2.2), and the
                 second-order exponential Runge-Kutta step built on it (the
                 higher-order extension section 1 mentions);
* ``diagnostics`` labels from 8-bit scan intensities (section 3.1 thresholds,
                 sampled at the stencil points as in section 3.5), the tumour
                 volume (section 3.5) and the largest distance between tumour
                 points (section 3.2);
* ``adjoint``    discrete adjoint (gradients of 0.5||u_T - u_target||^2 with
                 respect to u0, rho and the class diffusivities) and central
                 finite differences.
"""

from . import operator, plan, integrator, reference, adjoint, rosenbrock, exprk2, diagnostics  # noqa: F401
