"""Plain, slow, float64 CPU oracle for pairwise-perturbation CP-ALS.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library never
imports, links or calls anything here, and this package imports nothing from
the GPU library.  The two share only the seeded input generators in
``tensorgen``.

Contents (each function cites the passage of the paper it follows):

* ``oracle.cp``      -- MTTKRP by its elementwise definition, the explicit
                        unfolding x Khatri-Rao form, partially contracted
                        intermediates, CP-ALS sweep (Algorithm 1), fit.
* ``oracle.pp``      -- pairwise perturbation operators, the approximated
                        right-hand side (equation for the general PP update),
                        PP-CP-ALS control (Algorithm 3), the reinterpreted
                        pairwise ALS (Algorithm 5).
* ``oracle.linalg``  -- Cholesky solve of the normal equations.
* ``oracle.bf16``    -- bfloat16 round-to-nearest-even emulation.
* ``oracle.tree``    -- dimension-tree schedules and their flop counts
                        (Section 2.5 and Section 3.2.3).
* ``oracle.mlp``     -- float64 two-layer MLP forward/backward/Adam used to
                        check the learned PP controller.
"""
from . import bf16, cp, linalg, mlp, pp, tree  # noqa: F401
