"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test would fail for a plausible mistake in ``oracle/``: a wrong corner or
interior entry of K_j or M_j, a wrong ABC sign, a transposed Kronecker factor, a
wrong band layout, a non-pivoting or mis-indexed solve.
"""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import fem, eigen


def _theta_neumann(n):
    return np.pi * np.arange(n) / (n - 1)


def _fe_dispersion(theta, h):
    # Generalised eigenvalue of the 3-point FE stencils (1/h)[-1 2 -1] and
    # (h/6)[1 4 1] on the mode e^{i k theta}: (2-2cos)/h / ((h/6)(4+2cos)).
    return 6.0 * (1.0 - np.cos(theta)) / (h * h * (2.0 + np.cos(theta)))


@pytest.mark.parametrize("n", [5, 8, 33])
def test_neumann_pencil_closed_form(n):
    """Both faces Neumann: the cosine modes cos(k pi i/(n-1)) are exact
    eigenvectors, so eig(K, M) = 6(1-cos t)/(h^2 (2+cos t)), t = k pi/(n-1)."""
    h = 1.0 / (n - 1)
    K = fem.stiffness_1d(n, h, 7.0, False, False)
    M = fem.mass_1d(n, h)
    lam = np.sort(sla.eigvals(K, M).real)
    ref = np.sort(_fe_dispersion(_theta_neumann(n), h))
    assert np.max(np.abs(lam - ref)) <= 1e-10 * ref.max()


@pytest.mark.parametrize("n", [6, 17])
def test_dirichlet_interior_closed_form(n):
    """The interior block (rows/cols 1..n-2) is the Dirichlet pencil: its
    eigenvalues are the same dispersion relation at t = k pi/(n-1), k=1..n-2.
    This pins the interior entries independently of the corners."""
    h = 1.0 / (n - 1)
    K = fem.stiffness_1d(n, h, 3.0, True, True)[1:-1, 1:-1]
    M = fem.mass_1d(n, h)[1:-1, 1:-1]
    lam = np.sort(sla.eigvals(K, M).real)
    ref = np.sort(_fe_dispersion(_theta_neumann(n)[1:-1], h))
    assert np.max(np.abs(lam - ref)) <= 1e-10 * ref.max()


def test_abc_corner_entries_and_symmetry():
    n, h, w = 9, 1.0 / 8, 5.0
    K = fem.stiffness_1d(n, h, w, True, False)
    assert K[0, 0] == pytest.approx((1 - 1j * w * h) / h)
    assert K[-1, -1] == pytest.approx(1 / h)
    assert np.array_equal(K, K.T)
    M = fem.mass_1d(n, h)
    assert M[0, 0] == pytest.approx(2 * h / 6) and M[4, 4] == pytest.approx(4 * h / 6)
    assert M[3, 4] == pytest.approx(h / 6)
    # row sums: K annihilates constants in the interior (consistency), M sums to h
    assert np.allclose(K[1:-1].sum(1), 0)
    assert np.allclose(M.sum(1)[1:-1], h)


@pytest.mark.parametrize("n", [8, 13])
def test_periodic_pencil_dft_diagonalises(n):
    """Circulant K^B, M^B: the DFT matrix F[l,i] = e^{-2 pi i l i/n}
    diagonalises them with the closed-form symbols, and the generalised
    eigenvalues are the dispersion relation at t = 2 pi l/n."""
    h = 1.0 / (n - 1)
    KB, MB = eigen.periodic_pencil(n, h)
    F = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    Fi = np.conj(F) / n
    t = 2 * np.pi * np.arange(n) / n
    DK = F @ KB @ Fi
    DM = F @ MB @ Fi
    assert np.max(np.abs(DK - np.diag((2 - 2 * np.cos(t)) / h))) < 1e-12 / h
    assert np.max(np.abs(DM - np.diag(h / 6 * (4 + 2 * np.cos(t))))) < 1e-14
    lam = np.sort(sla.eigvals(KB, MB).real)
    assert np.allclose(lam, np.sort(_fe_dispersion(t, h)), rtol=1e-10, atol=1e-8)


def _grid_params(grid, omega, abc):
    h = tuple(1.0 / (n - 1) for n in grid)
    return grid, h, omega, abc


def test_operator_symmetric_not_hermitian():
    grid, h, w, abc = _grid_params((7, 6), 4.0, ((True, True), (True, False)))
    A = fem.operator(grid, h, w, abc)
    assert abs(A - A.T).max() == 0.0
    assert abs(A - A.conj().T).max() > 0.0
    grid3 = (4, 5, 3)
    A3 = fem.operator(grid3, tuple(1.0 / (n - 1) for n in grid3), 2.5, ((True,) * 2,) * 3)
    assert abs(A3 - A3.T).max() == 0.0


def test_interior_9point_stencil():
    """Bilinear elements on a square mesh: 3*stiffness stencil is
    [[-1,-1,-1],[-1,8,-1],[-1,-1,-1]] and 36/h^2 * mass stencil is
    [[1,4,1],[4,16,4],[1,4,1]]."""
    n, w = 7, 3.0
    grid = (n, n)
    h = (1.0 / (n - 1),) * 2
    A = fem.operator(grid, h, w, ((True, True), (True, True))).toarray()
    i, j = 3, 2
    row = A[i * n + j].reshape(n, n)[i - 1:i + 2, j - 1:j + 2]
    stiff = np.array([[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]]) / 3.0
    mass = np.array([[1, 4, 1], [4, 16, 4], [1, 4, 1]]) * h[0] ** 2 / 36.0
    assert np.allclose(row, stiff - w * w * mass, atol=1e-14)
    assert np.count_nonzero(A[i * n + j]) == 9


def test_interior_27point_stencil():
    """Trilinear elements on a cubic mesh: stiffness stencil 8h/3 (centre),
    0 (faces), -h/6 (edges), -h/12 (corners); mass (h^3/216)*{64,16,4,1}."""
    n, w = 6, 2.0
    grid = (n, n, n)
    hh = 1.0 / (n - 1)
    A = fem.operator(grid, (hh,) * 3, w, ((True, True),) * 3).toarray()
    c = (2, 3, 2)
    row = A[(c[0] * n + c[1]) * n + c[2]].reshape(n, n, n)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for d in (-1, 0, 1):
                k = abs(a) + abs(b) + abs(d)
                stiff = {0: 8 * hh / 3, 1: 0.0, 2: -hh / 6, 3: -hh / 12}[k]
                mass = {0: 64, 1: 16, 2: 4, 3: 1}[k] * hh ** 3 / 216
                assert row[c[0] + a, c[1] + b, c[2] + d] == pytest.approx(stiff - w * w * mass, abs=1e-13)


@pytest.mark.parametrize("grid,abc", [
    ((5, 4), ((True, True), (True, True))),
    ((9, 7), ((True, False), (False, True))),
    ((4, 5, 3), ((True, True), (True, True), (True, True))),
    ((3, 4, 6), ((True, False), (True, True), (False, True))),
])
def test_banded_solve_and_apply_vs_dense(grid, abc):
    """Brute force on tiny grids: dense np.linalg.solve of the assembled A, and
    the dense product A u, must agree with the banded LU and the matrix-free
    product."""
    g, h, w, abc = _grid_params(grid, 3.7, abc)
    A = fem.operator(g, h, w, abc).toarray()
    N = A.shape[0]
    rng = np.random.default_rng(5)
    f = rng.standard_normal((2, N)) + 1j * rng.standard_normal((2, N))
    u = fem.solve(g, h, w, abc, f)
    ud = np.linalg.solve(A, f.T).T
    assert np.max(fem.rel_error(u, ud)) < 1e-12
    assert np.max(np.abs(fem.apply(g, h, w, abc, f) - (A @ f.T).T)) < 1e-12 * np.abs(A).max() * 10
    assert np.max(fem.rel_residual(g, h, w, abc, u, f)) < 1e-13
    # band width is tight: the outermost band is non-zero, nothing lies beyond
    bw = fem.bandwidth(g)
    assert np.abs(np.diag(A, bw)).max() > 0
    if bw + 1 < N:
        assert np.abs(np.diag(A, bw + 1)).max() == 0


def _phi_coeffs(w):
    # phi(t) = 1 + a1 t + a2 t^2 + t^3 with phi'(0) = -i w phi(0) and
    # phi'(1) = i w phi(1): the 1D profile satisfies the first-order ABC
    # (eq. (1st-order-abc), outward normal -x at 0 and +x at 1) exactly.
    a1 = -1j * w
    a2 = (w * w + 3j * w - 3) / (2 - 1j * w)
    return a1, a2


def _manufactured(grid, w):
    """Load vector and nodal exact solution for u* = prod_j phi(x_j):
    f = -Lap u* - w^2 u*, f_i = integral f psi_i (weak form, eq.
    (helmholtzWeak)), assembled exactly by 1D Gauss moments."""
    a1, a2 = _phi_coeffs(w)
    phi = lambda t: 1 + a1 * t + a2 * t * t + t ** 3
    ddphi = lambda t: 2 * a2 + 6 * t + 0 * t
    h = [1.0 / (n - 1) for n in grid]
    P = [fem.hat_moments(n, hh, phi) for n, hh in zip(grid, h)]
    D = [fem.hat_moments(n, hh, ddphi) for n, hh in zip(grid, h)]
    d = len(grid)

    def outer(vs):
        out = vs[0]
        for v in vs[1:]:
            out = np.multiply.outer(out, v)
        return out

    f = -w * w * outer(P)
    for j in range(d):
        vs = [D[k] if k == j else P[k] for k in range(d)]
        f = f - outer(vs)
    xs = [np.linspace(0, 1, n) for n in grid]
    u_exact = outer([phi(x) for x in xs])
    return f.ravel(), u_exact.ravel(), tuple(h)


def test_phi_satisfies_abc():
    w = 2 * np.pi
    a1, a2 = _phi_coeffs(w)
    phi = lambda t: 1 + a1 * t + a2 * t * t + t ** 3
    dphi = lambda t: a1 + 2 * a2 * t + 3 * t * t
    assert abs(-dphi(0.0) - 1j * w * phi(0.0)) < 1e-12
    assert abs(dphi(1.0) - 1j * w * phi(1.0)) < 1e-12


def test_manufactured_convergence_2d():
    """O(h^2) nodal convergence at omega = 2 pi (the paper's wavenumber). A
    wrong ABC sign or corner, a wrong Kronecker factor or a wrong load would
    stall the error at O(1) or O(h)."""
    w = 2 * np.pi
    errs = []
    for n in (17, 33, 65, 129):
        f, ue, h = _manufactured((n, n), w)
        u = fem.solve((n, n), h, w, ((True, True), (True, True)), f)
        errs.append(np.max(np.abs(u - ue)) / np.max(np.abs(ue)))
    rates = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.6 < r < 4.4 for r in rates[1:]), (errs, rates)
    assert errs[-1] < 1e-3


def test_manufactured_convergence_3d():
    w = 2 * np.pi
    errs = []
    for n in (5, 9, 17):
        f, ue, h = _manufactured((n, n, n), w)
        u = fem.solve((n, n, n), h, w, ((True, True),) * 3, f)
        errs.append(np.max(np.abs(u - ue)) / np.max(np.abs(ue)))
    rates = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert rates[-1] > 3.3, (errs, rates)


@pytest.mark.parametrize("n,ppw", [(16, 10.0), (65, 10.0), (128, 8.0)])
def test_abc_eigen_oracle_invariants(n, ppw):
    """Pins of the dense eigen-oracle by identities the pencil must satisfy:
    K V = M V diag(lam), V^T M V = I, V^T K V = diag(lam), Im lam <= 0
    (v^H K v has imaginary part -w(|v_0|^2 + |v_{n-1}|^2) and M is SPD), and the
    trace identity sum(lam) = trace(M^{-1} K)."""
    h = 1.0 / (n - 1)
    w = 2 * np.pi * (n - 1) / ppw
    lam, V = eigen.abc_pencil(n, h, w)
    K = fem.stiffness_1d(n, h, w, True, True)
    M = fem.mass_1d(n, h)
    scale = np.abs(lam).max()
    assert np.max(np.abs(K @ V - M @ V * lam)) < 1e-10 * scale
    assert np.max(np.abs(V.T @ M @ V - np.eye(n))) < 1e-9
    assert np.max(np.abs(V.T @ K @ V - np.diag(lam))) < 1e-9 * scale
    assert lam.imag.max() < 0
    tr = np.trace(np.linalg.solve(M, K))
    assert abs(lam.sum() - tr) < 1e-10 * abs(tr)


def test_abc_eigen_oracle_neumann_limit():
    """With both faces Neumann the pencil is real and the oracle must return
    the closed-form cosine spectrum."""
    n = 40
    h = 1.0 / (n - 1)
    lam, V = eigen.abc_pencil(n, h, 9.0, False, False)
    assert np.allclose(np.sort(lam.real), np.sort(_fe_dispersion(_theta_neumann(n), h)),
                       rtol=1e-9, atol=1e-7)
    assert np.max(np.abs(lam.imag)) < 1e-8


def test_oracle_package_header_says_test_infrastructure():
    assert "TEST INFRASTRUCTURE ONLY" in oracle.__doc__
