"""Full-size workloads on the GPU, checked by properties the CPU oracle can
evaluate at any size: the relative residual ||f - A u|| / ||f|| computed by the
oracle's own matrix-free operator (complex128, numpy/scipy), and agreement of
the FP64 and the mixed-precision refined solutions.  Banded LU is infeasible
here (about 3.3 TB of band at 4096^2)."""

import sys

import numpy as np
import pytest

from oracle import fem
from paper_1809_03808_amd import helm, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _solve(wl, precision, nrhs=None):
    grid, omega = wl["grid"], wl["omega"]
    nrhs = nrhs or wl["nrhs"]
    h = inputs.spacing(grid)
    mask = (1 << (2 * len(grid))) - 1
    seeds = [inputs.rhs_seed(wl["config"], 0, r) for r in range(nrhs)]
    f = inputs.gaussian_device(grid, seeds, "cuda")
    u = torch.empty_like(f)
    _say("full-size", grid, "prec", precision, "nrhs", nrhs)
    with helm.Plan(grid, h, omega, mask, precision=precision) as plan:
        rc = plan.solve(f, u, raise_on_error=False)
        rep = plan.report()
    torch.cuda.synchronize()
    _say("  report", rep)
    return rc, rep, f, u, h


def _abc(dim):
    return ((True, True),) * dim


def test_2d_4096_fp64_residual_by_oracle():
    wl = inputs.workload("2d_4096_ppw10")
    rc, rep, f, u, h = _solve(wl, helm.PREC_FP64)
    assert rc == helm.HELM_OK
    fc = f.cpu().numpy().reshape(1, -1)
    uc = u.cpu().numpy().reshape(1, -1)
    res = fem.rel_residual(wl["grid"], h, wl["omega"], _abc(2), uc, fc)
    _say("  oracle residual", res)
    assert res[0] <= 1e-10
    # the device FP64 residual agrees with the oracle's (to rounding when both
    # sit at the ~1e-14 floor)
    assert abs(res[0] - rep["rel_residual_max"]) <= 1e-2 * res[0] + 1e-14


def test_2d_4096_mixed_matches_fp64():
    wl = inputs.workload("2d_4096_ppw10")
    rc64, rep64, f, u64, h = _solve(wl, helm.PREC_FP64)
    rc32, rep32, f2, u32, _ = _solve(wl, helm.PREC_MIXED)
    assert rc64 == helm.HELM_OK and rc32 == helm.HELM_OK
    assert torch.equal(f, f2)
    d = (torch.linalg.vector_norm(u32 - u64) / torch.linalg.vector_norm(u64)).item()
    _say("  ||u_mixed - u_fp64|| / ||u_fp64|| =", d)
    assert rep32["rel_residual_max"] <= 1e-10
    assert d <= 1e-8


def test_3d_256_mixed_residual_by_oracle():
    wl = inputs.workload("3d_256_ppw10")
    rc, rep, f, u, h = _solve(wl, helm.PREC_MIXED)
    assert rc == helm.HELM_OK
    fc = f.cpu().numpy().reshape(1, -1)
    uc = u.cpu().numpy().reshape(1, -1)
    res = fem.rel_residual(wl["grid"], h, wl["omega"], _abc(3), uc, fc)
    _say("  oracle residual", res)
    assert res[0] <= 1e-10
