"""CPU oracle for the mixed-precision HODLR matrix-vector product.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, fp64 restatement of
what the method computes, written from the paper (Carson, Chen, Liu, "Mixed
Precision HODLR Matrices", arXiv 2407.21637).  It exists to check the HIP
library and nothing else: only the test suite, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.
The product (``paper_2407_21637_amd``) never imports it, and it never imports
the product; the two share no code.  The only common module is
``hodlr_inputs``, which holds seeded input generators and none of the
method's arithmetic.

Modules, each citing the passage it follows:

* ``formats``  -- unit roundoffs (Table 1.1) and round-to-nearest-even codecs
                  that simulate storage in a lower precision (Sect. 4 setup,
                  precisions simulated by rounding).
* ``tree``     -- the cluster tree (Def. 2.1), the practical ceil split
                  (Sect. 4 setup) and the canonical off-diagonal block list
                  (eq. (2.1)).
* ``construct``-- dense truncated-SVD construction of an eps-HODLR matrix
                  (Def. 2.3, eq. (3.1)).
* ``assign``   -- the adaptive precision rule (Alg. "Adaptive-precision
                  HODLR Format", eq. (3.3)).
* ``quantize`` -- storing a level's generators in its precision (Alg.
                  "Mixed-precision HODLR Format"), with per-column power-of-2
                  scales for the narrow formats.
* ``matvec``   -- HODLR_MATVEC (Alg. "HODLR_MATVEC"), its absolute-value
                  twin and a dense assembly of the stored operator.
* ``lowp``     -- the product in a low working precision (bf16, fp16): the
                  Thm. 3.5 / Sect. 4 setting with u = u_W, operands rounded
                  to W, and its componentwise tolerance.
* ``bounds``   -- the error bounds of Thm. 3.1 / eqs. (3.4)-(3.7) and
                  Thm. 3.5, and the componentwise tolerance used to compare
                  the GPU result with this oracle.

Parity pinned: every function here is checked by ``tests/test_oracle_*.py``
against values and facts that do not come from the oracle itself (library
casts, brute force, closed forms, the paper's printed constants and bounds).
"""
