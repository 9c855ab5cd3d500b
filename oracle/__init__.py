"""Plain FP64 CPU oracle of the hierarchical ORAS + randomised-SVD coarse solver.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
GPU library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library itself never does.
It shares no code with the library: it is written in NumPy/SciPy, step by step
in the order the paper gives the method, without blocking or fusion.

Modules
-------
operator   the discrete impedance Helmholtz operator of a box (eq. (lap1) in
           Sec. 1 and the free-space problem of Sec. 3.1), the right-hand side
           and the sparse direct solve.
geometry   the hierarchical overlapping decomposition (Sec. 1, Sec. 3 set-up):
           boxes, restricted prolongations, interface nodes, neighbours.
schwarz    local solvers, the interface map T_i and its randomised SVD
           (Sec. 2), the coarse basis C and A_c = C^H A C (eq. (coarse1)), the
           two-level ORAS step (eqs. (sub1)-(coarse1)) and the recursion of the
           hierarchy (Sec. 1, Sec. 2).
krylov     the outer loops: stationary iteration and right-preconditioned
           restarted (F)GMRES (Sec. 3).

Parity pins: every function is pinned by a test under ``tests/`` marked
``not gpu``; see the header of each module for the pin of each part.
"""

from . import operator, geometry, schwarz, krylov  # noqa: F401
