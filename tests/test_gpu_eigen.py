"""Device eigen-setup (helm_eig1d_device, HELM_EIGEN_DEVICE) against the dense
QZ eigen-oracle and the reduction oracle, against the host setup at the
paper's and the benchmark's lengths, and end to end: plans built with either
setup solve alike, and the device-built plans meet the banded-LU oracle."""

import numpy as np
import pytest

from oracle import eigen, fem
from paper_1809_03808_amd import helm, inputs

pytestmark = pytest.mark.gpu


def _match(lam_a, lam_b):
    """Pair each eigenvalue of a with the nearest of b; (perm, max rel err)."""
    perm = np.array([np.argmin(np.abs(lam_b - x)) for x in lam_a])
    assert len(set(perm.tolist())) == len(lam_a), "eigenvalues did not pair one-to-one"
    err = np.max(np.abs(lam_a - lam_b[perm]) / np.abs(lam_b[perm]).clip(1.0))
    return perm, err


def _rows_agree(vb, V0, V1, tol):
    """Boundary rows up to each column's sign: sign-free products."""
    scale = np.max(np.abs(V0)) ** 2
    assert np.max(np.abs(vb[0] * vb[1] - V0 * V1)) < tol * scale
    assert np.max(np.abs(vb[0] ** 2 - V0 ** 2)) < tol * scale
    assert np.max(np.abs(vb[1] ** 2 - V1 ** 2)) < tol * scale


@pytest.mark.parametrize("n,ppw,lo,hi", [
    (3, 10.0, True, True), (8, 10.0, True, True), (33, 10.0, True, True), (64, 8.0, True, True),
    (128, 10.0, True, True), (256, 20.0, True, True), (100, 12.0, True, False),
    (65, 9.0, False, True), (40, 10.0, False, False), (129, 4.0, True, True),
])
def test_device_eigenpairs_match_qz_oracle(n, ppw, lo, hi):
    h = 1.0 / (n - 1)
    w = 2 * np.pi * (n - 1) / ppw
    lam, vb = helm.eig1d(n, h, w, lo, hi, device=True)
    lam_o, V_o = eigen.abc_pencil(n, h, w, lo, hi)
    perm, err = _match(lam, lam_o)
    assert err < 1e-10, err
    _rows_agree(vb, V_o[0, perm], V_o[-1, perm], 1e-8)
    assert np.all(np.diff(lam.real) >= 0)  # sorted by real part


@pytest.mark.parametrize("n,omega", [(513, 2 * np.pi), (1025, 2 * np.pi * 102.4), (1024, 2 * np.pi * 102.3)])
def test_device_eigenpairs_match_reduction_oracle(n, omega):
    h = 1.0 / (n - 1)
    lam, vb = helm.eig1d(n, h, omega, device=True)
    lam_o, V_o = eigen.abc_pencil_by_reduction(n, h, omega)
    perm, err = _match(lam, lam_o)
    assert err < 1e-10, err
    _rows_agree(vb, V_o[0, perm], V_o[-1, perm], 1e-8)


@pytest.mark.parametrize("n,ppw,lo,hi", [
    (512, 10.0, True, True), (1025, 10.0, True, True), (2049, 10.0, True, True), (4096, 10.0, True, True),
    (2049, None, True, True), (1000, 10.0, True, False), (777, 12.0, False, True),
])
def test_device_matches_host_setup(n, ppw, lo, hi):
    """The host setup refines in extended precision and the device one in
    double-double arithmetic: both round the same eigenvalues to FP64."""
    h = 1.0 / (n - 1)
    w = 2 * np.pi if ppw is None else 2 * np.pi * (n - 1) / ppw
    lam_d, vb_d = helm.eig1d(n, h, w, lo, hi, device=True)
    lam_h, vb_h = helm.eig1d(n, h, w, lo, hi)
    rel = np.abs(lam_d - lam_h) / np.abs(lam_h).clip(1.0)
    assert rel.max() < 1e-14, rel.max()
    _rows_agree(vb_d, vb_h[0], vb_h[1], 1e-12)


def _solve(plan, f):
    import torch
    u = torch.empty_like(f)
    plan.solve(f, u)
    torch.cuda.synchronize()
    return u.cpu().numpy()


@pytest.mark.parametrize("grid,ppw,prec,extra", [
    ((300, 257), 10.0, helm.PREC_FP64, {}),
    ((257, 129), 8.0, helm.PREC_MIXED, {}),
    ((64, 48), 10.0, helm.PREC_FP64, {"transform": helm.TRANSFORM_DENSE}),
    ((33, 40, 9), 6.0, helm.PREC_FP64, {"boundary": helm.BOUNDARY_TABLES}),
    ((24, 20, 17), 6.0, helm.PREC_MIXED, {"boundary": helm.BOUNDARY_LINES}),
    ((16, 12, 9), 5.0, helm.PREC_FP64, {"transform": helm.TRANSFORM_DENSE}),
])
def test_plans_from_either_setup_agree(grid, ppw, prec, extra):
    import torch
    h = inputs.spacing(grid)
    w = 2 * np.pi * (max(grid) - 1) / ppw
    f = inputs.gaussian_device(grid, [inputs.rhs_seed(9, 1, r) for r in range(2)], "cuda")
    u_d = _solve(helm.Plan(grid, h, w, precision=prec, eigen=helm.EIGEN_DEVICE, **extra), f)
    u_h = _solve(helm.Plan(grid, h, w, precision=prec, eigen=helm.EIGEN_HOST, **extra), f)
    rel = np.linalg.norm((u_d - u_h).ravel()) / np.linalg.norm(u_h.ravel())
    assert rel < 1e-11, rel
    # and the device-built plan against the banded-LU oracle
    if np.prod(grid) <= 80000:
        fh = f.cpu().numpy().reshape(2, -1)
        ref = fem.solve(grid, h, w, ((True, True),) * len(grid), fh)
        err = np.linalg.norm(u_d.reshape(2, -1) - ref) / np.linalg.norm(ref)
        assert err < (1e-9 if prec == helm.PREC_FP64 else 1e-8), err
