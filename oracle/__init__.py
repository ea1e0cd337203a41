"""Plain FP64 CPU reference for the Tucker-compressed VSIE coupling matvec.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the GPU library; both draw
their synthetic inputs from ``workloads`` alone.

Contents (each function cites the passage of the paper it follows):

* ``fields``     closed-form point-current columns of the E-field operator
                 (eq. 2 with the Green's function of eq. 3); PWC and PWL
                 voxel bases (Sec. II.A.1).
* ``hosvd``      n-mode products (eq. 7), the Tucker model (eq. 6) and the
                 truncated HOSVD (Sec. II.B.1).
* ``matvec``     Algorithm 1 (Y = Z X) and Algorithm 2 (Y = Z^* X) of
                 Sec. III.B, single-entry decompression (Sec. III.C), dense
                 truth, the least-squares loss and its gradient.
* ``accounting`` memory and operation counts of Tables II and III.
* ``aca``        adaptive cross approximation with partial pivoting, dense
                 or with U compressed column by column (Algorithm 3), and
                 the ACA + Tucker products (Sec. II.B.2, III.B, III.C).

Parity status: every function is pinned by the ``-m "not gpu"`` tests against
closed forms, theorems, brute force or numbers printed in the paper, except
the field values of specific geometries, which the paper never prints
(parity unpinned beyond the closed-form and invariant checks).
"""
from . import aca, accounting, fields, hosvd, matvec  # noqa: F401
