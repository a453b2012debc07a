"""CPU oracle for the FFT-based fast direct Helmholtz solver (Toivanen & Wolfmayr,
"A fast Fourier transform based direct solver for the Helmholtz problem").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_1809_03808_amd``): no kernels, tables, constants or helpers.

What it computes, in complex128:

* ``fem``   -- the bilinear / trilinear finite-element system A u = f of
  Section 2 (1D stiffness and mass matrices, eqs. (matrixK), (matrixM); the
  Kronecker operator, eqs. (A2D), (A3D)), its direct solution by banded LU with
  partial pivoting (LAPACK zgbsv), the matrix-free product A u and the residual
  f - A u.  The fast solver is a *direct* method (Section 3.1: Steps 1-3 are an
  exact identity), so its result is exactly A^{-1} f up to rounding; this
  module is that plain definition.
* ``eigen`` -- the dense generalized eigenproblem K_1 V_1 = M_1 V_1 Lambda^A_1
  of eq. (EVP1a) with the normalisation V^T M V = I of eq. (EVPcondA), solved by
  QZ (scipy.linalg.eig), or for long axes by the flip-symmetry split and a
  Cholesky reduction to LAPACK zgeev; and the periodic auxiliary matrices of
  eqs. (matrixKper), (matrixMper).
* ``sov``   -- a second direct solver for grids whose band is too wide for
  banded LU: dense separation of variables with the absorbing-boundary
  eigenvectors (eqs. (A2Dinv), (A3Dinv)) and one pivoted tridiagonal solve
  (LAPACK zgtsv) per mode, optionally refined with the residual of ``fem``.

Each function is pinned by tests under ``tests/test_oracle_*.py`` against facts
that do not come from the oracle itself: brute-force dense solves on tiny grids,
banded LU against the separation of variables and vice versa, QZ against the
reduced eigenproblems,
closed-form eigenvalues of the Neumann, Dirichlet and periodic 1D pencils,
exact symmetry of A, the closed-form interior 9-point stencil, and O(h^2)
convergence to a manufactured solution that satisfies the absorbing boundary
condition exactly.  Parity against numbers printed in the paper is unpinned:
the paper prints timings only, no solution values, errors or residuals.
"""

from . import fem, eigen, sov  # noqa: F401
