"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package builds sparse symmetric matrices (lower triangle, CSC, 0-based,
int64 indices, rows sorted inside each column, diagonal present) and the
geometric nested-dissection permutation passed to the analysis step.  It holds
none of the selected-inversion arithmetic: no factorization, no inverse, no
symbolic analysis of the Cholesky/LDL^T structure.  Both the oracle and the
HIP path consume exactly the arrays produced here.

The paper measures on DFT Hamiltonians (H - zS type, from DGDFT and SIESTA)
and on UFL collection matrices (Table 1, Section 4).  Those files are not
available, so the regular-grid problems below stand in for them: weighted 3-D
Laplacians for the nd-class UFL matrices and shifted complex-symmetric
operators for the DFT pole-expansion matrices.
"""

from .grids import (  # noqa: F401
    Workload,
    nested_dissection,
    laplacian_2d_dirichlet,
    weighted_laplacian_3d,
    gmrf_2d,
    stencil27_complex,
    shifted_batch,
    random_pattern,
    config,
    CONFIG_NAMES,
)
