"""Plain FP64 CPU oracle for the Vanka-smoothed shifted-Laplacian Helmholtz solver.

TEST INFRASTRUCTURE ONLY.  This package is a slow, obviously-correct NumPy/SciPy
restatement of the method of Yovel, He and Treister, "Vanka-smoothed Shifted
Laplacian multigrid preconditioners for the Helmholtz equations" (2025).  It exists
to check the HIP library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never does, and
this package never imports the product package.  It shares no code with the HIP
path: operators are built from 1D Kronecker factors and sparse matrices, patch
inverses with ``numpy.linalg.inv``, the coarsest solve with ``scipy.linalg.lu_factor``.

Modules
    discretization  the Helmholtz operator, absorbing layer and the shift (Sec. 1, 2.1, 2.3)
    intergrid       restriction / prolongation families (Sec. 3.1)
    hierarchy       Galerkin coarse operators and operator complexity (Sec. 3.1)
    vanka           additive Vanka patches, weights and the smoother (Sec. 3.2, 3.3)
    cycle           two-grid / V / W cycles (Sec. 2.2, Algorithm "Two-grid cycle")
    krylov          right-preconditioned flexible GMRES(m) (Sec. 2.3)
    lfa             local Fourier analysis symbols (Sec. 2.4, 4)

Parity status: every module is pinned by CPU tests against closed forms, dense
brute force or values printed in the paper, except where a docstring says
"parity unpinned".
"""
