"""Plain, slow, FP64 CPU oracle for compressed threshold pivoting.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import anything from this package.
The product path (the HIP library and its Python binding) never imports,
calls or links it, and the two share no code.

Modules:
    threshold  -- the pivot search of Section 2 on a trapezoid [A11; R],
                  with the strict / relaxed / restricted variants of
                  Sections 3.2 and 4, a decision log with margins, forced
                  decisions and exact rational arithmetic.
    supernode  -- compression (eq. (4.2), Section 4.2), Factor + Solve of a
                  supernode, Form (the Schur complement), closed forms.
    dense      -- dense LDL^T by panels with carried delays, the solve with
                  the factors, the backward error and iterative refinement.

Parity unpinned: the loop-control reading (pass restart) and the order of
the interchanges for a 2x2 pivot are fixed only by this implementation; no
value printed in the paper checks them beyond internal consistency.
"""

from . import threshold, supernode, dense  # noqa: F401
