"""Sketch-preconditioned mixed-precision least squares on one MI355X (gfx950).

The method (Carson and Dauzickaite): sketch [A b] with a Gaussian embedding
(Algorithm 1), take the R factor of a Householder QR of the sketch, run
LSQR right-preconditioned with R from the sketch-and-solve point
(Algorithm 2) and refine x and r on the augmented system with
split-preconditioned FGMRES (Algorithm 2's refinement loop).  All of it runs in libls.so
(hand-written HIP); this package is its Python binding.
"""

from .api import (  # noqa: F401
    Solver,
    iter_opts,
    ls_lsir_gmres,
    ls_lsqr_precond,
    ls_omega,
    ls_philox,
    ls_qr_r,
    ls_sketch,
    ls_solve,
    ls_solve_batched,
    precs,
    problem,
    qr_workspace_size,
    sketch_opts,
    sketch_plan_info,
    sketch_split_rows,
    sketch_terms_for,
    workspace,
    workspace_size,
)
from ._binding import LsError, load  # noqa: F401
