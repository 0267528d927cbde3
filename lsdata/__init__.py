"""Seeded synthetic least-squares inputs shared by the tests, the benchmark
and the oracle checks.

This module only *builds input data*; it contains none of the solver's
arithmetic (no sketch, no QR of a sketch, no LSQR, no refinement).  Both the
GPU library and the CPU oracle receive the arrays it returns, so the two
sides see identical inputs without sharing any of the method's code.
"""

from .problems import (  # noqa: F401
    Problem,
    WORKLOADS,
    data_seed,
    make_problem,
    make_paper_problem,
    make_batch_sizes,
)
