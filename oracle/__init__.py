"""CPU oracle for the sketch-preconditioned least-squares method.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package; only the test-suite, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
library: the two see the same seeded inputs (from ``lsdata``) and nothing
else.

What is here (plain numpy, float64 unless a step says otherwise):

* ``philox``  -- Philox4x32-10 (Salmon et al., SC'11) and the Box-Muller
  Gaussian stream that defines the sketch operator Omega (Section 2: Gaussian
  embedding with N(0, 1/s) entries).
* ``formats`` -- round-to-nearest-even into bf16 / fp16 / OCP e4m3, the
  power-of-two column scaling of Section 3.2, and the split of A into a sum
  of narrow-format terms.
* ``sketch``  -- Algorithm 1, the sketch: Y = Omega [A b].
* ``qr``      -- Algorithm 1, the QR: economic Householder QR, R factor only;
  back substitution with R and R^T.
* ``lsqr``    -- Algorithm 2, the LSQR solve: right-preconditioned with R,
  started at the sketch-and-solve solution (Paige and Saunders, 1982).
* ``lsir``    -- Algorithm 2, the refinement loop: augmented-system refinement with
  split-preconditioned flexible GMRES.
* ``refsolve`` -- the exact solution of the stored data (extended-precision
  residual refinement on the augmented system), the target of every
  forward-error figure (Section 5 measures against a 64-digit solution).
* ``solve``   -- the whole pipeline, and condition-number helpers used by
  the checks of Section 4.1.
"""

from . import philox, formats, sketch, qr, lsqr, lsir, refsolve, solve  # noqa: F401
