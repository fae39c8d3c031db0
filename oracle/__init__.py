"""FP64 CPU oracle for the Green's-function Poisson convolution.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never calls it, and this package shares
no code with that path: no kernels, tables, constants or helpers.

What it computes is the plain definition of the method's result (paper,
Section 2, Eqs. 2-3 with the zero padding of free axes): the discrete
convolution of the density with the Green's function on the grid padded to
S_j = N_j B_j (Section 3), done with whole-grid FP64 FFTs and no zero-skipping,
axis ordering or fusion.  The Green's functions themselves are not given in
the paper; `greens` states the reading used and every constant it needs.
"""

from .greens import (  # noqa: F401
    C2_LOG_ORIGIN,
    C3_COULOMB_ORIGIN,
    EULER_GAMMA,
    kernel_fourier,
    kernel_octant,
    mixed_kernel,
    padded_shape,
)
from .solve import brute_force, real_space_kernel, rel_l2, solve  # noqa: F401
from . import isf  # noqa: F401
