"""Dense separation of variables: a second CPU oracle for grids whose band is
too wide for banded LU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The absorbing-boundary eigenvectors diagonalise the operator along the
periodised axes (Section 4.1.1, eq. (A2Dinv); Section 5.1.1, eq. (A3Dinv)):
with K_j V_j = M_j V_j Lambda_j and V_j^T M_j V_j = I (eqs. (EVP1a),
(EVPcondA)),

    2D: (V_1^T (x) I) A (V_1 (x) I) = blockdiag_l ((lambda_{1,l} - w^2) M_2 + K_2)
    3D: (V_1^T (x) V_2^T (x) I) A (V_1 (x) V_2 (x) I)
        = blockdiag_{l,m} ((lambda_{1,l} + lambda_{2,m} - w^2) M_3 + K_3),

so u = (V (x) I) T^{-1} (V^T (x) I) f with one tridiagonal solve per mode
along the last axis.  The eigenpairs come from ``eigen`` (QZ for short axes,
the reduction of ``abc_pencil_by_reduction`` for long ones), the dense
transforms are plain matrix products, and each tridiagonal system is solved
by LAPACK zgtsv (Gaussian elimination with partial pivoting).  Nothing here
uses the periodic auxiliary problem or the three steps of Section 3.1, so an
error in those is not shared.
"""

import numpy as np
from scipy.linalg import lapack

from . import eigen, fem
from .fem import mass_1d, stiffness_1d

QZ_MAX = 512  # above this length the eigenpairs come from the reduction


def axis_eigenpairs(n, h, omega, lo, hi):
    """(lam, V) of the 1D pencil of one periodised axis, V^T M V = I."""
    if n <= QZ_MAX:
        return eigen.abc_pencil(n, h, omega, lo, hi)
    return eigen.abc_pencil_by_reduction(n, h, omega, lo, hi)


def _diagonals(T):
    """(sub, main, super) diagonals of a tridiagonal matrix."""
    return (np.ascontiguousarray(np.diag(T, -1)), np.ascontiguousarray(np.diag(T)),
            np.ascontiguousarray(np.diag(T, 1)))


def _line_solve(sig, M, K, rhs):
    """(sig M + K) z = rhs for one tridiagonal line matrix (zgtsv); M and K
    are given by their diagonals (``_diagonals``)."""
    dl = sig * M[0] + K[0]
    d = sig * M[1] + K[1]
    du = sig * M[2] + K[2]
    _, _, _, x, info = lapack.zgtsv(dl, d, du, rhs)
    if info != 0:
        raise ArithmeticError(f"zgtsv info {info}")
    return x


def solve(grid, h, omega, abc, f, eig=None, refine=0):
    """u = A^{-1} f for one right-hand side f (shape (N,) or grid), complex128.
    ``abc`` as in ``fem``; ``eig`` optionally supplies the eigenpairs of the
    periodised axes (a list of (lam, V)) so that several right-hand sides
    share them.  ``refine`` > 0 adds that many steps of classical iterative
    refinement u <- u + S(f - A u), S this solver, with the residual from
    the oracle's matrix-free operator (``fem.residual``); the eigenvectors of
    long axes carry errors of order cond(V) * 1e-16, which one step removes."""
    grid = tuple(int(n) for n in grid)
    if eig is None:
        eig = [axis_eigenpairs(grid[j], h[j], omega, abc[j][0], abc[j][1]) for j in range(len(grid) - 1)]
    u = _solve_once(grid, h, omega, abc, f, eig)
    for _ in range(refine):
        r = fem.residual(grid, h, omega, abc, u, np.asarray(f).reshape(-1))
        u = u + _solve_once(grid, h, omega, abc, r, eig)
    return u


def solve_refined(grid, h, omega, abc, f, eta_tol=1e-15, max_steps=4):
    """``solve`` followed by refinement steps until the normwise backward error
    of u (``fem.backward_error``) is at most ``eta_tol``, or ``max_steps``
    steps.  Near-resonant modes (small |lambda - w^2| on long axes) amplify
    the eigenvector errors, so one step is not always enough.  The relative
    residual is not the criterion: for loads that make ||A|| ||u|| much larger
    than ||f|| (the paper's load, near resonance) its rounding floor lies well
    above 1e-13 for any FP64 solver, banded LU included.  Returns
    (u, backward error, steps taken)."""
    grid = tuple(int(n) for n in grid)
    eig = [axis_eigenpairs(grid[j], h[j], omega, abc[j][0], abc[j][1]) for j in range(len(grid) - 1)]
    f = np.asarray(f, dtype=np.complex128).reshape(-1)
    nf = np.linalg.norm(f)
    nA = fem.norm_bound(grid, h, omega, abc)
    u = _solve_once(grid, h, omega, abc, f, eig)
    steps = 0
    while True:
        r = fem.residual(grid, h, omega, abc, u, f)
        eta = float(np.linalg.norm(r) / (nA * np.linalg.norm(u) + nf))
        if eta <= eta_tol or steps >= max_steps:
            return u, eta, steps
        u = u + _solve_once(grid, h, omega, abc, r, eig)
        steps += 1


def _solve_once(grid, h, omega, abc, f, eig):
    d = len(grid)
    F = np.asarray(f, dtype=np.complex128).reshape(grid)
    nL = grid[-1]
    KL = _diagonals(stiffness_1d(nL, h[-1], omega, abc[-1][0], abc[-1][1]))
    ML = _diagonals(mass_1d(nL, h[-1]).astype(np.complex128))
    w2 = omega * omega
    if d == 2:
        lam1, V1 = eig[0]
        G = V1.T @ F                                   # (V_1^T (x) I) f
        Z = np.empty_like(G)
        for l in range(grid[0]):
            Z[l] = _line_solve(lam1[l] - w2, ML, KL, G[l])
        return (V1 @ Z).reshape(-1)                     # (V_1 (x) I) z
    (lam1, V1), (lam2, V2) = eig
    n1, n2, n3 = grid
    G = (V1.T @ F.reshape(n1, n2 * n3)).reshape(n1, n2, n3)   # along x_1
    G = np.matmul(V2.T[None], G)                               # along x_2, per x_1 mode
    Z = np.empty_like(G)
    for l in range(n1):
        for m in range(n2):
            Z[l, m] = _line_solve(lam1[l] + lam2[m] - w2, ML, KL, G[l, m])
    del G
    U = np.matmul(V2[None], Z)
    del Z
    U = (V1 @ U.reshape(n1, n2 * n3)).reshape(-1)
    return U
