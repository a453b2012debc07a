"""Finite-element Helmholtz system of Section 2 and its direct banded solve.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain complex128 code,
no blocking or fusion: every function is the definition it cites.

Conventions
-----------
* ``grid``  -- node counts (n_1, ..., n_d), d = 2 or 3; nodes x_{j,i} = i*h_j.
* ``h``     -- mesh sizes (h_1, ..., h_d); the paper uses h_j = 1/(n_j - 1).
* ``abc``   -- per axis a pair (lo, hi) of faces.  A boolean face is True for
  the first-order absorbing boundary condition (eq. (1st-order-abc)) and
  False for Neumann (eq. (Neumannbc)); a number g makes the face a Robin
  (impedance) face du/dn + g u = 0 with outward normal n, the other
  separable boundary conditions of Section 1.  The absorbing condition is the
  case g = -i omega, Neumann g = 0.
* ``c``     -- the zeroth-order coefficient of -Lap u - c u = f (Section 1
  allows either sign); None means c = omega^2, the Helmholtz operator.
* Vectors are C-ordered with x_1 the slowest axis, i.e. the Kronecker ordering
  of eqs. (A2D), (A3D): the node (i_1, ..., i_d) sits at flat index
  ((i_1 * n_2) + i_2) * n_3 + i_3.
"""

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# 1D matrices, Section 2, eqs. (matrixK) and (matrixM)
# ---------------------------------------------------------------------------

def face_coefficient(omega, face):
    """g of a face in du/dn + g u = 0 (outward normal): a boolean face is the
    first-order absorbing condition du/dn - i omega u = 0 (eq.
    (1st-order-abc), g = -i omega) or Neumann (g = 0); a number is g itself."""
    if isinstance(face, (bool, np.bool_)):
        return -1j * omega if face else 0.0
    return complex(face)


def zeroth_order(omega, c=None):
    """The coefficient c of -Lap u - c u: omega^2 unless given."""
    return omega ** 2 if c is None else c


def stiffness_1d(n, h, omega, abc_lo, abc_hi):
    """K_j of eq. (matrixK): (1/h) tridiag(-1, 2, -1) with corner entries
    k/h, k = 1 - i*omega*h on an absorbing face and k = 1 on a Neumann face
    (the corner values stated right after eq. (matrixM)); a Robin face adds
    its boundary term g u v, k = 1 + g h.  Dense complex."""
    K = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        K[i, i] = 2.0
        if i > 0:
            K[i, i - 1] = -1.0
        if i < n - 1:
            K[i, i + 1] = -1.0
    K[0, 0] = 1.0 + h * face_coefficient(omega, abc_lo)
    K[n - 1, n - 1] = 1.0 + h * face_coefficient(omega, abc_hi)
    return K / h


def mass_1d(n, h):
    """M_j of eq. (matrixM): (h/6) tridiag(1, 4, 1) with corners 2.  Dense real."""
    M = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        M[i, i] = 4.0
        if i > 0:
            M[i, i - 1] = 1.0
        if i < n - 1:
            M[i, i + 1] = 1.0
    M[0, 0] = 2.0
    M[n - 1, n - 1] = 2.0
    return M * (h / 6.0)


def _axis_pair(grid, h, omega, abc, j):
    K = sp.csr_matrix(stiffness_1d(grid[j], h[j], omega, abc[j][0], abc[j][1]))
    M = sp.csr_matrix(mass_1d(grid[j], h[j]).astype(np.complex128))
    return K, M


# ---------------------------------------------------------------------------
# The Kronecker operator, Section 2, eqs. (A2D) and (A3D)
# ---------------------------------------------------------------------------

def operator(grid, h, omega, abc, c=None):
    """Sparse A.  2D: A = (K1 - w^2 M1) (x) M2 + M1 (x) K2            (A2D)
                   3D: A = (K1 - w^2 M1) (x) M2 (x) M3
                           + M1 (x) (K2 (x) M3 + M2 (x) K3)            (A3D)
    with c in place of w^2 when given."""
    d = len(grid)
    K1, M1 = _axis_pair(grid, h, omega, abc, 0)
    K2, M2 = _axis_pair(grid, h, omega, abc, 1)
    S1 = K1 - zeroth_order(omega, c) * M1
    if d == 2:
        A = sp.kron(S1, M2) + sp.kron(M1, K2)
    elif d == 3:
        K3, M3 = _axis_pair(grid, h, omega, abc, 2)
        A = sp.kron(sp.kron(S1, M2), M3) + sp.kron(M1, sp.kron(K2, M3) + sp.kron(M2, K3))
    else:
        raise ValueError("dimension must be 2 or 3")
    A = sp.csr_matrix(A)
    A.eliminate_zeros()  # sparse kron stores the zero entries of its dense blocks
    return A


def bandwidth(grid):
    """Half bandwidth of A in the x_1-slowest ordering: the farthest coupled
    node of a 9- (27-) point stencil is one step along every axis."""
    if len(grid) == 2:
        return grid[1] + 1
    return grid[1] * grid[2] + grid[2] + 1


def to_banded(A, bw):
    """LAPACK/scipy diagonal-ordered storage ab[bw + i - j, j] = A[i, j]."""
    A = sp.coo_matrix(A)
    keep = A.data != 0
    A = sp.coo_matrix((A.data[keep], (A.row[keep], A.col[keep])), shape=A.shape)
    n = A.shape[0]
    ab = np.zeros((2 * bw + 1, n), dtype=np.complex128)
    ab[bw + A.row - A.col, A.col] = A.data
    return ab


def operator_in_order(grid, h, omega, abc, perm, c=None):
    """A with its unknowns numbered with the axes in the order ``perm``
    (slowest first): the same Kronecker terms as eqs. (A2D), (A3D), each
    term's 1D factors taken in that order.  perm = (0, ..., d-1) is
    ``operator``; any other order is a symmetric permutation P A P^T of it."""
    d = len(grid)
    pairs = [_axis_pair(grid, h, omega, abc, j) for j in range(d)]
    K = [k for k, _ in pairs]
    M = [m for _, m in pairs]
    S1 = K[0] - zeroth_order(omega, c) * M[0]
    if d == 2:
        terms = [(S1, M[1]), (M[0], K[1])]
    elif d == 3:
        terms = [(S1, M[1], M[2]), (M[0], K[1], M[2]), (M[0], M[1], K[2])]
    else:
        raise ValueError("dimension must be 2 or 3")
    A = None
    for t in terms:
        T = t[perm[0]]
        for j in perm[1:]:
            T = sp.kron(T, t[j])
        A = T if A is None else A + T
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    return A


def narrowest_order(grid):
    """Axis order (slowest first) with the smallest half bandwidth: the
    longest axis slowest, the shortest fastest."""
    return tuple(sorted(range(len(grid)), key=lambda j: (-grid[j], j)))


def solve(grid, h, omega, abc, f, order=None, c=None):
    """u = A^{-1} f by banded LU with partial pivoting (LAPACK zgbsv via
    scipy.linalg.solve_banded), complex128.  ``f`` has shape (N,) or
    (nrhs, N), C-ordered with x_1 slowest; the result has the same shape.

    The band is stored in the unknown numbering of ``order`` (default: the
    narrowest, see ``narrowest_order``); renumbering the unknowns is a
    symmetric permutation, so the solution is the same vector, and a grid
    with a long last axis keeps a narrow band."""
    grid = tuple(int(n) for n in grid)
    d = len(grid)
    perm = tuple(order) if order is not None else narrowest_order(grid)
    f = np.asarray(f, dtype=np.complex128)
    F = np.atleast_2d(f).reshape((-1,) + grid)
    nr = F.shape[0]
    Fp = F.transpose((0,) + tuple(j + 1 for j in perm)).reshape(nr, -1)
    gp = tuple(grid[j] for j in perm)
    A = operator_in_order(grid, h, omega, abc, perm, c)
    bw = bandwidth(gp)
    ab = to_banded(A, bw)
    up = sla.solve_banded((bw, bw), ab, Fp.T, overwrite_ab=True, check_finite=True).T
    inv = np.argsort(perm)
    U = up.reshape((nr,) + gp).transpose((0,) + tuple(int(j) + 1 for j in inv))
    U = np.ascontiguousarray(U).reshape(nr, -1)
    return U if f.ndim == 2 else U[0]


# ---------------------------------------------------------------------------
# Matrix-free product and residual (the operator of eqs. (A2D), (A3D))
# ---------------------------------------------------------------------------

def _along(T, U, axis):
    """Apply the 1D sparse matrix T along ``axis`` of the array U:
    (I (x) ... (x) T (x) ... (x) I) vec(U)."""
    Um = np.moveaxis(U, axis, 0)
    shp = Um.shape
    out = (T @ Um.reshape(shp[0], -1)).reshape(shp)
    return np.moveaxis(out, 0, axis)


def apply(grid, h, omega, abc, u, c=None):
    """A u without forming A, using (X (x) Y) vec(U) = vec(X U Y^T) axis by axis.
    ``u`` has shape (N,) or (nrhs, N)."""
    d = len(grid)
    u = np.asarray(u, dtype=np.complex128)
    lead = u.shape[:-1]
    U = u.reshape(lead + tuple(grid))
    off = len(lead)
    pairs = [_axis_pair(grid, h, omega, abc, j) for j in range(d)]
    K1, M1 = pairs[0]
    S1 = K1 - zeroth_order(omega, c) * M1
    if d == 2:
        K2, M2 = pairs[1]
        AU = _along(M2, _along(S1, U, off), off + 1) + _along(K2, _along(M1, U, off), off + 1)
    else:
        K2, M2 = pairs[1]
        K3, M3 = pairs[2]
        M1U = _along(M1, U, off)
        AU = (_along(M3, _along(M2, _along(S1, U, off), off + 1), off + 2)
              + _along(M3, _along(K2, M1U, off + 1), off + 2)
              + _along(K3, _along(M2, M1U, off + 1), off + 2))
    return AU.reshape(u.shape)


def residual(grid, h, omega, abc, u, f, c=None):
    """r = f - A u (complex128)."""
    return np.asarray(f, dtype=np.complex128) - apply(grid, h, omega, abc, u, c)


def rel_residual(grid, h, omega, abc, u, f, c=None):
    """Per right-hand side ||f - A u||_2 / ||f||_2 over all nodes."""
    r = residual(grid, h, omega, abc, u, f, c)
    f = np.asarray(f)
    return np.linalg.norm(np.atleast_2d(r), axis=-1) / np.linalg.norm(np.atleast_2d(f), axis=-1)


def norm_bound(grid, h, omega, abc, c=None):
    """Upper bound of ||A||_2 from the Kronecker form of eqs. (A2D), (A3D):
    A is symmetric, so ||A||_2 <= ||A||_inf, and the triangle inequality with
    ||X (x) Y||_inf = ||X||_inf ||Y||_inf bounds ||A||_inf by the sum over the
    terms of the products of the 1D factors' row-sum norms."""
    d = len(grid)
    K = [stiffness_1d(grid[j], h[j], omega, abc[j][0], abc[j][1]) for j in range(d)]
    M = [mass_1d(grid[j], h[j]) for j in range(d)]
    ni = lambda X: float(np.max(np.sum(np.abs(X), axis=1)))  # noqa: E731
    S1 = ni(K[0] - zeroth_order(omega, c) * M[0])
    nK = [ni(x) for x in K]
    nM = [ni(x) for x in M]
    if d == 2:
        return S1 * nM[1] + nM[0] * nK[1]
    return S1 * nM[1] * nM[2] + nM[0] * nK[1] * nM[2] + nM[0] * nM[1] * nK[2]


def backward_error(grid, h, omega, abc, u, f, c=None):
    """Normwise backward error ||f - A u|| / (||A|| ||u|| + ||f||) per right-hand
    side (2-norms, ||A|| from ``norm_bound``): the size of the smallest
    relative perturbation of A and f of which u is the exact solution, up to
    the bound on ||A||.  A backward-stable direct solve makes it a small
    multiple of the unit roundoff whatever the conditioning, whereas the
    relative residual ||f - A u|| / ||f|| also grows with ||A|| ||u|| / ||f||."""
    r = np.atleast_2d(residual(grid, h, omega, abc, u, f, c))
    u = np.atleast_2d(u)
    f = np.atleast_2d(f)
    nA = norm_bound(grid, h, omega, abc, c)
    return np.linalg.norm(r, axis=-1) / (nA * np.linalg.norm(u, axis=-1) + np.linalg.norm(f, axis=-1))


def rel_error(u, u_ref):
    """Per right-hand side ||u - u_ref||_2 / ||u_ref||_2."""
    u = np.atleast_2d(u)
    u_ref = np.atleast_2d(u_ref)
    return np.linalg.norm(u - u_ref, axis=-1) / np.linalg.norm(u_ref, axis=-1)


# ---------------------------------------------------------------------------
# Consistent load vector of a smooth source (weak form, eq. (helmholtzWeak))
# ---------------------------------------------------------------------------

_GAUSS3_X = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
_GAUSS3_W = np.array([5.0, 8.0, 5.0]) / 9.0


def hat_moments(n, h, g):
    """b_i = integral over [0, (n-1)h] of g(t) psi_i(t) dt for the 1D hat
    functions psi_i, with 3-point Gauss-Legendre per element (exact when g is a
    polynomial of degree <= 4)."""
    b = np.zeros(n, dtype=np.complex128)
    for e in range(n - 1):
        a = e * h
        for xg, wg in zip(_GAUSS3_X, _GAUSS3_W):
            t = a + 0.5 * h * (xg + 1.0)
            w = 0.5 * h * wg
            s = (t - a) / h
            gv = g(t)
            b[e] += w * gv * (1.0 - s)
            b[e + 1] += w * gv * s
    return b
