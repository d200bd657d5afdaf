"""Plain CPU oracle for the rank-local work of a persistent neighborhood
all-to-all-v halo exchange (MPI Advance, Sec. 2.2).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the
package smoke check and the benchmark's CPU-baseline leg may import, call or
execute anything in this package.  It shares no code with the HIP library
(``paper_2309_07337_amd``) and never imports it; the only module both sides use
is the seeded input generator (``workloads``).

Contents (each function cites the passage it follows):

* ``plan``  : halo discovery, owner segmentation, send-list transpose, the
              locality-aware 2-step plan (node dedup + on-node redistribution)
              and the transpose CSR used by the backward.
* ``cpu``   : ctypes loader of ``cpu_move.c``, the same pack / gather /
              fixed-order transpose sum as plain OpenMP loops (the all-cores
              CPU baseline of the benchmark), pinned by
              ``tests/test_cpu_oracle.py``.
* ``move``  : pack, simulated transfer, redistribution pack, unpack, the
              fixed-order transpose sum (backward), the backward taken
              through the plan's stages, and the plain definitions they must
              reproduce (direct global gather, closed-form adjoint).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against brute force on tiny inputs, closed forms of the stencil workloads,
invariants (symmetry, conservation, exactly-once delivery, dedup = unique
count), special cases (one rank per node == plain; one node == no
inter-node traffic; the staged backward of the plain plan == the closed-form
adjoint) and, for the staged backward's summation order, a symbolic brute
force written from the reading alone.  No function is "parity unpinned".
"""
from . import plan, move  # noqa: F401
