"""Seeded synthetic least-squares problems shared by the oracle-side tests and the GPU-side tests.

This module generates inputs only; it holds none of the solver's arithmetic.  Both the CPU oracle
(``oracle/``) and the HIP path read the bytes it produces.

Construction (paper, Section 1, the 4000 x 50 test problem of Figure 1 and the problems of
Section 5): ``A = U diag(sigma) V^T`` with Haar-distributed orthonormal ``U`` (m x n) and ``V``
(n x n), singular values ``sigma_i = 10^{p_i}`` with ``p_i`` equally spaced from 0 to
``-log10(kappa)``, a Gaussian solution ``x_true`` and a residual ``r_perp`` drawn uniformly from
the sphere of the requested radius inside the orthogonal complement of ``range(A)``; then
``b = A x_true + r_perp``.
"""

from .problems import (  # noqa: F401
    Problem,
    make_problem,
    make_multi_problem,
    make_problem_torch,
    log_spaced_sigma,
    haar_cholqr2,
    ComplexProblem,
    make_complex_problem,
    make_prony_problem,
    prony_samples,
)
