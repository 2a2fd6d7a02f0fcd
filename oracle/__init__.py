"""FP64 CPU oracle for the matrix power kernel -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct reference that the HIP
path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product package never
does, and it shares no code with the HIP path (it imports nothing from
``paper_2309_02228_amd``; inputs come from the separate ``synth`` generators).

Everything is written from the paper's statement of the method
(Alappat, Thies, Hager, Fehske, Wellein: "Algebraic temporal blocking for
sparse iterative solvers on multi-core CPUs"):

* ``spmv``, ``mpk``                 -- Sec. 3, Alg. 1 and Alg. 2
* ``round_values``                  -- reduced-precision storage of the matrix
  values (reading R11; the paper itself works in FP64)
* ``round_values_bf16_rowscale``    -- BF16 values with a per-row FP32 scale
  (reading R16)
* ``chebyshev_inverse_coeffs``      -- the degree-d Chebyshev polynomial
  preconditioner (Sec. 5; reading R12)
* ``refine_solve``                  -- FP64 iterative refinement around it, with
  FP32-stored values for the corrections (reading R13; beyond the paper)
* ``newton_basis``                  -- Sec. 4 (Newton basis of the s-step method)
* ``poly_monomial``/``poly_newton``  -- Sec. 5.2, Eq. (3)
* ``poly_chebyshev``                -- Sec. 5.3 (Chebyshev smoother; the
  three-term recurrence itself is not printed in the paper)
* ``pattern_graph``, ``bfs_levels``,
  ``level_permutation``,
  ``permute_symmetric``             -- Sec. 3 (BFS level structure of the
  matrix graph) and Sec. 5.1.2 (levels come from A alone)
* ``group_levels``, ``wavefront_schedule``, ``validate_schedule``,
  ``run_schedule``                  -- Sec. 3 (level groups from the cache size
  and the skewed wavefront over them), readings R14 and R15
* ``leja_order``, ``newton_shifts``, ``cholqr_truncated``, ``sstep_cycle``,
  ``sstep_gmres``                   -- Sec. 4 (s-step GMRES, Alg. 3a/3c: Newton
  basis, BOrtho, TSQR) with the right polynomial preconditioner of Sec. 5,
  readings R17-R19
* ``diagonal``, ``jacobi_precondition``, ``jacobi_mpk`` -- Sec. 5.1 (Jacobi
  preconditioner, k iterations from zero) in the right-preconditioned MPK,
  reading R20
* ``spmv_lower``, ``gs2_precondition``, ``gs2_mpk`` -- Sec. 5.1 (two-stage
  Gauss-Seidel, one outer iteration from zero, gamma inner sweeps) in the
  right-preconditioned MPK, reading R21
* ``gs2_smooth_residual`` -- Sec. 5.3, the AMG pre-smoother (outer GS2 sweeps in the
  non-compact form, gamma = 0: Jacobi) followed by the residual the cycle needs next,
  reading R23
* ``arnoldi``, ``ritz_shifts`` -- Sec. 4, Newton shifts from the Ritz values of a few
  standard Arnoldi (GMRES) steps, reading R24
* ``interval_shifts``, ``sstep_gmres_precond`` -- s-step GMRES without a
  preconditioner or with the diagonal (Jacobi) one, a blocked Newton MPK per
  block of s vectors, reading R22

* ``ref_c`` (``mpk_ref.c``)         -- the same MPK in plain C, single-threaded
  and with OpenMP over rows (the CPU baselines of the benchmark), equal to
  ``mpk`` bitwise

Parity status of each function is stated in its docstring.  The readings
taken where the paper is silent are listed in ``mpk_oracle.READINGS``.
"""
from .mpk_oracle import *  # noqa: F401,F403
from .mpk_oracle import READINGS  # noqa: F401
