"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package only *generates inputs*: tissue label volumes, class
diffusivities, initial tumour densities and the parameters of the standard
workloads.  It holds none of the method's arithmetic (no operator, no time
stepping), so both the CPU oracle and the HIP path can be fed from it without
sharing any computation.

The paper's runs use a private MRI head (section 3.1); these synthetic heads
stand in for it with the same grid shape, tissue classes and coefficients
(Table 1: white matter 0.13, gray matter 0.013, air 0 mm^2/day, rho = 0.025/day).
"""

from .head import (  # noqa: F401
    CLASS_D_PAPER,
    Head,
    gaussian_blob,
    make_head,
    uniform_box,
)
from .configs import (  # noqa: F401
    Workload,
    BatchInstance,
    c1_plain,
    c2_head,
    c3_batch,
    c4_adjoint,
    c5_separable,
)
