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


def abc_pencil_by_reduction(n, h, omega, abc_lo=True, abc_hi=True):
    """The same eigenpairs as ``abc_pencil`` (eq. (EVP1a), V^T M V = I), for
    lengths where dense QZ is too slow (about 90 s at n = 1024 and growing as
    n^3), by textbook reductions to standard eigenproblems:

    1. when both faces carry the same condition, the pencil commutes with the
       flip J (node i <-> node n-1-i), so with the orthonormal even / odd
       vectors (e_i +- e_{n-1-i})/sqrt(2) it splits into two pencils of about
       n/2 (the coupling block vanishes; checked to rounding);
    2. each block pencil (K_b, M_b) with M_b real symmetric positive definite
       becomes the complex symmetric matrix C = L^{-1} K_b L^{-T},
       M_b = L L^T (Cholesky), whose eigenpairs come from LAPACK zgeev;
    3. v = S L^{-T} y, scaled to v^T M v = 1 (plain transpose, eq. (EVPcondA)).

    Returns (lam, V) sorted by (Re, Im) of the eigenvalue like ``abc_pencil``."""
    K = stiffness_1d(n, h, omega, abc_lo, abc_hi)
    M = mass_1d(n, h)
    half = n // 2
    if bool(abc_lo) == bool(abc_hi):
        cols_e, cols_o = [], []
        s = 1.0 / np.sqrt(2.0)
        for i in range(half):
            e = np.zeros(n)
            e[i] = s
            e[n - 1 - i] = s
            cols_e.append(e)
            o = np.zeros(n)
            o[i] = s
            o[n - 1 - i] = -s
            cols_o.append(o)
        if n % 2:
            e = np.zeros(n)
            e[half] = 1.0
            cols_e.append(e)
        blocks = [np.array(cols_e).T, np.array(cols_o).T]
        cross = blocks[0].T @ K @ blocks[1]
        if np.max(np.abs(cross)) > 1e-13 * np.max(np.abs(K)):
            raise ArithmeticError("flip symmetry broken: even/odd blocks couple")
    else:
        blocks = [np.eye(n)]
    lams, vecs = [], []
    for S in blocks:
        Kb = S.T @ K @ S
        Mb = S.T @ M @ S
        L = np.linalg.cholesky(Mb)
        Li = sla.solve_triangular(L, np.eye(L.shape[0]), lower=True)
        C = Li @ Kb @ Li.T
        w, Y = np.linalg.eig(C)
        V = S @ (Li.T @ Y)
        lams.append(w)
        vecs.append(V)
    lam = np.concatenate(lams)
    V = np.concatenate(vecs, axis=1)
    s = np.sqrt(np.sum(V * (M @ V), axis=0))  # v_l^T M v_l
    V = V / s
    order = np.lexsort((lam.imag, lam.real))
    return lam[order], V[:, order]
