"""Dense 1D eigenproblems of Section 3.2.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``abc_pencil`` -- K_1 V_1 = M_1 V_1 Lambda^A_1 (eq. (EVP1a)), solved by QZ
  (scipy.linalg.eig on the dense pencil), each column scaled by
  1 / (v^T M v)^{1/2} so that V^T M V = I and V^T K V = Lambda (eqs. (EVPcondA),
  (sA), (sAnorm): plain transpose, because the pencil is complex symmetric).
* ``periodic_pencil`` -- the circulant K^B, M^B of eqs. (matrixKper),
  (matrixMper), built entry by entry.
"""

import numpy as np
import scipy.linalg as sla

from .fem import stiffness_1d, mass_1d


def abc_pencil(n, h, omega, abc_lo=True, abc_hi=True):
    """Return (lam, V) for the 1D pencil (K, M) of eqs. (matrixK), (matrixM),
    with V normalised by V^T M V = I.  Eigenpairs are sorted by (Re, Im) of the
    eigenvalue; the sign of each column is arbitrary (only products of two
    entries of a column are determined)."""
    K = stiffness_1d(n, h, omega, abc_lo, abc_hi)
    M = mass_1d(n, h)
    lam, V = sla.eig(K, M)
    s = np.sqrt(np.einsum("il,ij,jl->l", V, M, V))
    V = V / s
    order = np.lexsort((lam.imag, lam.real))
    return lam[order], V[:, order]


def periodic_pencil(n, h):
    """Circulant K^B, M^B of eqs. (matrixKper), (matrixMper) (dense, real)."""
    KB = np.zeros((n, n))
    MB = np.zeros((n, n))
    for i in range(n):
        KB[i, i] = 2.0 / h
        MB[i, i] = 4.0 * h / 6.0
        for j in ((i - 1) % n, (i + 1) % n):
            KB[i, j] = -1.0 / h
            MB[i, j] = h / 6.0
    return KB, MB
