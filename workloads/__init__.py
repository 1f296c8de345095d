"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This package only *describes* problems: it builds the sparse test Hamiltonians
(as CSR arrays and as stencil descriptors), the Gaussian-well potentials and the
random start blocks C_0.  It contains none of the eigensolver's arithmetic, and
it imports neither the oracle nor the GPU package.
"""

from .problems import (  # noqa: F401
    Problem,
    StencilSpec,
    laplacian_2d_dirichlet_csr,
    periodic_fd_csr,
    gaussian_wells,
    start_block,
    make_problem,
    config_problem,
    serving_stream,
    serving_problem,
    CONFIGS,
    GenProblem,
    fem_problem,
)
