"""Pins of the oracle's general operator: Robin (impedance) faces
du/dn + g u = 0 and a zeroth-order coefficient c of either sign,
-Lap u - c u = f (the separable boundary conditions and zeroth-order terms
Section 1 allows).  The absorbing condition is the face g = -i omega."""

import numpy as np
import pytest

from oracle import eigen, fem


def test_boolean_faces_are_the_absorbing_and_neumann_cases():
    n, h, w = 9, 0.125, 7.0
    K_abc = fem.stiffness_1d(n, h, w, True, False)
    K_num = fem.stiffness_1d(n, h, w, -1j * w, 0.0)
    assert np.array_equal(K_abc, K_num)


@pytest.mark.parametrize("g_lo,g_hi", [(0.0, 0.0), (2.5, 0.0), (0.7, 3.1), (1.5 - 4j, -2j), (-3j, 0.25)])
def test_boundary_form_of_constants(g_lo, g_hi):
    """1^T K 1 is the integral of |grad 1|^2 (zero) plus the boundary terms
    g_lo + g_hi of the weak form; 1^T M 1 is the length of the interval."""
    n, h = 13, 1.0 / 12
    K = fem.stiffness_1d(n, h, 3.0, g_lo, g_hi)
    one = np.ones(n)
    assert abs(one @ K @ one - (g_lo + g_hi)) < 1e-12
    assert abs(one @ fem.mass_1d(n, h) @ one - 1.0) < 1e-14


@pytest.mark.parametrize("grid", [(6, 5), (4, 5, 3)])
def test_neumann_laplace_annihilates_constants(grid):
    """c = 0 with Neumann faces: A 1 = 0 (the singular case)."""
    h = tuple(1.0 / (n - 1) for n in grid)
    abc = ((False, False),) * len(grid)
    N = int(np.prod(grid))
    Au = fem.apply(grid, h, 5.0, abc, np.ones(N), c=0.0)
    assert np.max(np.abs(Au)) < 1e-12
    A = fem.operator(grid, h, 5.0, abc, c=0.0)
    assert np.max(np.abs(A @ np.ones(N))) < 1e-12


def test_modified_helmholtz_with_robin_faces_is_positive_definite():
    """c < 0 and real g >= 0: A is real symmetric positive definite."""
    grid, h = (7, 6), (1.0 / 6, 1.0 / 5)
    abc = ((0.5, 0.0), (2.0, 1.0))
    A = fem.operator(grid, h, 1.0, abc, c=-9.0).toarray()
    assert np.max(np.abs(A.imag)) == 0.0
    assert np.max(np.abs(A - A.T)) < 1e-14
    assert np.linalg.eigvalsh(A.real).min() > 0


def test_robin_pencil_is_real_and_positive():
    """K v = lambda M v with real g > 0: real positive eigenvalues (symmetric
    positive definite pencil), V^T M V = I, and K V = M V Lambda."""
    n, h = 40, 1.0 / 39
    lam, V = eigen.abc_pencil(n, h, 1.0, 3.0, 0.5)
    K = fem.stiffness_1d(n, h, 1.0, 3.0, 0.5)
    M = fem.mass_1d(n, h)
    assert np.max(np.abs(lam.imag)) < 1e-9 * np.max(np.abs(lam))
    assert lam.real.min() > 0
    assert np.max(np.abs(V.T @ M @ V - np.eye(n))) < 1e-10
    assert np.max(np.abs(K @ V - M @ V * lam)) < 1e-9 * np.max(np.abs(lam))


def _phi_coeffs(g_lo, g_hi):
    """phi(t) = 1 + a1 t + a2 t^2 + t^3 with -phi'(0) + g_lo phi(0) = 0 and
    phi'(1) + g_hi phi(1) = 0: the 1D profile satisfies the Robin condition
    du/dn + g u = 0 on both ends (outward normal -x at 0, +x at 1)."""
    a1 = g_lo
    a2 = -(a1 + 3 + g_hi * (2 + a1)) / (2 + g_hi)
    return a1, a2


def _manufactured(grid, faces, c):
    """Load vector and nodal exact solution for u* = prod_j phi_j(x_j):
    f = -Lap u* - c u*, f_i = integral f psi_i, exact by 1D Gauss moments."""
    h = [1.0 / (n - 1) for n in grid]
    P, D, U = [], [], []
    for (g_lo, g_hi), n, hh in zip(faces, grid, h):
        a1, a2 = _phi_coeffs(g_lo, g_hi)
        phi = lambda t, a1=a1, a2=a2: 1 + a1 * t + a2 * t * t + t ** 3
        ddphi = lambda t, a2=a2: 2 * a2 + 6 * t + 0 * t
        P.append(fem.hat_moments(n, hh, phi))
        D.append(fem.hat_moments(n, hh, ddphi))
        U.append(phi(np.linspace(0, 1, n)))

    def outer(vs):
        out = vs[0]
        for v in vs[1:]:
            out = np.multiply.outer(out, v)
        return out

    d = len(grid)
    f = -c * outer(P)
    for j in range(d):
        f = f - outer([D[k] if k == j else P[k] for k in range(d)])
    return f.ravel(), outer(U).ravel(), tuple(h)


def test_phi_satisfies_robin():
    for g_lo, g_hi in ((2.0, 0.5), (1 - 3j, -2j)):
        a1, a2 = _phi_coeffs(g_lo, g_hi)
        phi = lambda t: 1 + a1 * t + a2 * t * t + t ** 3
        dphi = lambda t: a1 + 2 * a2 * t + 3 * t * t
        assert abs(-dphi(0.0) + g_lo * phi(0.0)) < 1e-12
        assert abs(dphi(1.0) + g_hi * phi(1.0)) < 1e-12


@pytest.mark.parametrize("faces,c", [
    (((2.0, 0.5), (1.0, 3.0)), -40.0),            # modified Helmholtz, Robin
    (((0.0, 1.0), (0.5, 0.0)), 0.0),              # Laplace, Robin and Neumann
    (((1.0 - 6j, -6j), (-6j, 2.0 - 6j)), 36.0),   # Helmholtz, impedance faces
    (((-5j, -5j), (-5j, -5j)), -25.0),            # absorbing-type faces, c < 0
])
def test_manufactured_convergence_general(faces, c):
    """O(h^2) nodal convergence; a wrong sign of g or c, or a misplaced
    boundary term, stalls the error at O(1) or O(h)."""
    errs = []
    for n in (17, 33, 65, 129):
        f, ue, h = _manufactured((n, n), faces, c)
        u = fem.solve((n, n), h, 1.0, faces, f, c=c)
        errs.append(np.max(np.abs(u - ue)) / np.max(np.abs(ue)))
    rates = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.6 < r < 4.4 for r in rates[1:]), (errs, rates)


def test_manufactured_convergence_general_3d():
    faces, c = ((1.0, 0.0), (0.5, 2.0), (-4j, -4j)), -10.0
    errs = []
    for n in (5, 9, 17):
        f, ue, h = _manufactured((n, n, n), faces, c)
        u = fem.solve((n, n, n), h, 1.0, faces, f, c=c)
        errs.append(np.max(np.abs(u - ue)) / np.max(np.abs(ue)))
    rates = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert rates[-1] > 3.3, (errs, rates)
