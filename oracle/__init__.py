"""CPU oracle for the low-rank Lyapunov equation AX + XA^T + W = 0 (test infrastructure).

This package is test infrastructure only: it may be imported by the tests, by the smoke
check and by the benchmark's CPU-baseline leg, and by nothing on the product path.  It is
plain, slow, obviously-correct NumPy/SciPy code in float64 (lower precisions are emulated
where the paper's method asks for them) and shares no code with the GPU library.

Modules
  precision  -- Table 1.1 unit roundoffs and round-to-format ("chop") helpers.
  exact      -- the exact solution X by its plain definitions: the Kronecker system
                (eq 2.1), Bartels-Stewart on a complex Schur form, and the recurrence on a
                known real Schur form; closed forms for diagonal A and A = -alpha I.
  residual   -- the residual R(Z) / R(Z,Y) (eq 2.2, 2.17) and the normwise relative
                residual res of eq (4.1), formed densely in float64.
  signnewton -- the scaled sign-function Newton iteration: the dense form (eq 3.1), the
                factored Cholesky form (eq 3.2, Alg 3.1) and the factored LDL^T form
                (eq 3.3, Alg 3.2) with their rank truncations and the stopping rule (3.4).
  adjoint    -- gradients of tr(C X C^T) through the adjoint equation A^T Y + Y A + C^T C = 0.
  refine     -- the residual factorisations and solution updates (Fragments 2.1-2.4) and
                the mixed-precision IR loops (Alg 2.1, Alg 2.2) with the Section 4.1
                parameters and the stagnation test (4.2).

Parity pins for every function live in tests/test_oracle_*.py.
"""
from . import precision, exact, residual, signnewton, refine  # noqa: F401
