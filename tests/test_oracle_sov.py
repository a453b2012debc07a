"""Pins of the second CPU oracle (dense separation of variables, eq. (A2Dinv),
eq. (A3Dinv)), of the eigenpairs it uses for long axes, and of the banded
solve in a renumbered order.

Each check compares against something the function under test does not
compute itself: brute-force dense solves, banded LU of the assembled
operator, QZ on the dense pencil, and the defining identities K V = M V L,
V^T M V = I.  A dropped term, a transposed eigenvector matrix, a wrong mass
shift or a wrong axis order fails one of them.
"""

import numpy as np
import pytest

from oracle import eigen, fem, sov
from paper_1809_03808_amd import inputs


def _abc(dim, mask):
    return tuple(((mask >> (2 * j)) & 1 == 1, (mask >> (2 * j + 1)) & 1 == 1) for j in range(dim))


@pytest.mark.parametrize("grid,mask", [((5, 7), 0b1111), ((4, 3, 6), 0b110111), ((6, 5, 4), 0b111101),
                                       ((3, 16), 0b0111), ((7, 2 + 1, 9), 0b111111)])
def test_banded_solve_any_order_matches_dense(grid, mask):
    """Banded LU in the narrowest and in the natural unknown numbering equals
    a dense solve of the assembled operator (eqs. (A2D), (A3D))."""
    h = inputs.spacing(grid)
    abc = _abc(len(grid), mask)
    rng = np.random.default_rng(3)
    n = int(np.prod(grid))
    f = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    ud = np.linalg.solve(fem.operator(grid, h, 3.0, abc).toarray(), f.T).T
    for order in (None, tuple(range(len(grid))), tuple(reversed(range(len(grid))))):
        u = fem.solve(grid, h, 3.0, abc, f, order=order)
        assert np.max(np.abs(u - ud)) <= 1e-12 * np.max(np.abs(ud)), order


def test_operator_in_order_is_a_permutation():
    grid, abc = (4, 3, 5), _abc(3, 0b111011)
    h = inputs.spacing(grid)
    A = fem.operator(grid, h, 2.0, abc).toarray()
    perm = (2, 0, 1)
    B = fem.operator_in_order(grid, h, 2.0, abc, perm).toarray()
    idx = np.arange(int(np.prod(grid))).reshape(grid).transpose(perm).reshape(-1)
    assert np.max(np.abs(B - A[np.ix_(idx, idx)])) <= 1e-14 * np.max(np.abs(A))  # products in another order


@pytest.mark.parametrize("n,lo,hi", [(64, True, True), (65, True, True), (33, True, False),
                                     (40, False, False), (129, True, True)])
def test_eigen_reduction_matches_qz(n, lo, hi):
    """Flip split + Cholesky + zgeev gives QZ's eigenvalues and the same
    eigenvector outer products v_l v_l^T (the sign of a column is free)."""
    h = 1.0 / (n - 1)
    w = 2 * np.pi * (n - 1) / 10
    l1, V1 = eigen.abc_pencil(n, h, w, lo, hi)
    l2, V2 = eigen.abc_pencil_by_reduction(n, h, w, lo, hi)
    assert np.max(np.abs(l1 - l2)) <= 1e-12 * np.max(np.abs(l1))
    P1 = np.einsum("il,jl->ijl", V1, V1)
    P2 = np.einsum("il,jl->ijl", V2, V2)
    assert np.max(np.abs(P1 - P2)) <= 1e-9 * np.max(np.abs(P1))


@pytest.mark.parametrize("n", [1024, 1025])
def test_eigen_reduction_identities_long_axis(n):
    """At lengths where QZ is slow: K V = M V Lambda, V^T M V = I, all
    absorbing eigenvalues in the closed lower half plane, and their real
    parts spread over the FE spectrum [0, 12/h^2]."""
    h = 1.0 / (n - 1)
    w = 2 * np.pi * (n - 1) / 10
    lam, V = eigen.abc_pencil_by_reduction(n, h, w, True, True)
    K = fem.stiffness_1d(n, h, w, True, True)
    M = fem.mass_1d(n, h)
    R = K @ V - (M @ V) * lam
    assert np.max(np.abs(R)) <= 1e-8 * np.max(np.abs(lam)) * np.max(np.abs(M @ V))
    G = V.T @ M @ V
    assert np.max(np.abs(G - np.eye(n))) <= 1e-9
    assert np.max(lam.imag) <= 1e-9 * np.max(np.abs(lam))
    assert lam.real.min() > -1e-6 and lam.real.max() < 12.0 / h ** 2


CASES = [((9, 7), 0b1111, 5.0), ((8, 6), 0b1110, 4.0), ((12, 10), 0b0110, 9.0),
         ((6, 5, 4), 0b110111, 4.0), ((7, 8, 5), 0b111111, 6.0), ((5, 6, 7), 0b111100, 3.0)]


@pytest.mark.parametrize("grid,mask,omega", CASES)
def test_sov_matches_banded_lu(grid, mask, omega):
    h = inputs.spacing(grid)
    abc = _abc(len(grid), mask)
    f = inputs.gaussian(grid, 77).reshape(-1)
    ub = fem.solve(grid, h, omega, abc, f)
    us = sov.solve(grid, h, omega, abc, f)
    assert np.linalg.norm(us - ub) <= 1e-12 * np.linalg.norm(ub)


def test_sov_256sq_ppw10_matches_banded_lu():
    """2D 256 x 256 at 10 points per wavelength (band 257 wide): the dense
    separation of variables with one refinement step equals banded LU."""
    grid = (256, 256)
    h = inputs.spacing(grid)
    w = inputs.omega_for_ppw(256, 10.0)
    abc = _abc(2, 0b1111)
    f = inputs.gaussian(grid, 78).reshape(-1)
    ub = fem.solve(grid, h, w, abc, f)
    us = sov.solve(grid, h, w, abc, f, refine=1)
    assert np.linalg.norm(us - ub) <= 1e-12 * np.linalg.norm(ub)
    assert fem.rel_residual(grid, h, w, abc, us[None], f[None])[0] <= 1e-13


def test_sov_long_axis_uses_reduction_and_matches_banded_lu():
    """A periodised axis longer than the QZ limit (600 nodes) with a short
    line axis: the reduction's eigenpairs give banded LU's solution."""
    grid = (600, 5)
    h = inputs.spacing(grid)
    w = inputs.omega_for_ppw(600, 12.0)
    abc = _abc(2, 0b1111)
    f = inputs.gaussian(grid, 79).reshape(-1)
    assert grid[0] > sov.QZ_MAX
    ub = fem.solve(grid, h, w, abc, f)
    us = sov.solve(grid, h, w, abc, f, refine=1)
    assert np.linalg.norm(us - ub) <= 1e-12 * np.linalg.norm(ub)


def test_sov_refined_near_resonance_matches_banded_lu():
    """omega = 2 pi on a long axis with the paper's load (the paper's
    experiments): refined to a backward error at rounding level, the result
    equals banded LU to within the problem's conditioning."""
    grid = (1025, 9)
    h = inputs.spacing(grid)
    abc = _abc(2, 0b1111)
    f = inputs.paper_rhs(grid).reshape(-1)
    ub = fem.solve(grid, h, 2 * np.pi, abc, f)
    us, eta, steps = sov.solve_refined(grid, h, 2 * np.pi, abc, f)
    assert eta <= 1e-15
    assert abs(fem.backward_error(grid, h, 2 * np.pi, abc, us[None], f[None])[0] - eta) <= 1e-17
    assert np.linalg.norm(us - ub) <= 1e-10 * np.linalg.norm(ub)


@pytest.mark.parametrize("grid,mask,omega", [((9, 7), 0b1111, 5.0), ((6, 5, 4), 0b110111, 4.0),
                                             ((17, 12), 0b0110, 2 * np.pi)])
def test_norm_bound_and_backward_error(grid, mask, omega):
    """norm_bound bounds the exact ||A||_inf (and ||A||_2) from above within a
    small factor; banded LU has a backward error at rounding level, and a
    relative perturbation of size e of its solution one of order e."""
    import scipy.sparse.linalg as spl
    h = inputs.spacing(grid)
    abc = _abc(len(grid), mask)
    A = fem.operator(grid, h, omega, abc)
    nb = fem.norm_bound(grid, h, omega, abc)
    ninf = spl.norm(A, np.inf)
    n2 = np.linalg.norm(A.toarray(), 2)
    assert ninf <= nb * (1 + 1e-14) and n2 <= nb * (1 + 1e-14) and nb <= 4 * ninf
    f = inputs.gaussian(grid, 5).reshape(-1)
    u = fem.solve(grid, h, omega, abc, f)
    assert fem.backward_error(grid, h, omega, abc, u[None], f[None])[0] <= 1e-15
    rng = np.random.default_rng(6)
    up = u * (1 + 1e-9 * rng.standard_normal(u.size))
    eta = fem.backward_error(grid, h, omega, abc, up[None], f[None])[0]
    assert 1e-12 <= eta <= 1e-8
