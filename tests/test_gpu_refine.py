"""Refinement control and its failure paths (a tolerance that cannot be met,
a step that stops halving the residual), on the host loop of an eager solve,
on the device-controlled loop of a captured solve, and inside a batch graph.
In each case the report must say HELM_ENOCONV, and u must hold the last
iterate, whose oracle residual is the one reported."""

import sys

import numpy as np
import pytest

from oracle import fem
from paper_1809_03808_amd import helm, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


GRID, OMEGA = (64, 77), 35.0
ABC = ((True, True), (True, True))


def _data(seed):
    f = inputs.gaussian_batch(GRID, [seed, seed + 1])
    return f, torch.from_numpy(f).cuda()


def _oracle_res(u, f):
    return fem.rel_residual(GRID, inputs.spacing(GRID), OMEGA, ABC, u.reshape(2, -1), f.reshape(2, -1))


@pytest.mark.parametrize("prec,max_iter", [(helm.PREC_FP64, 2), (helm.PREC_MIXED, 2), (helm.PREC_FP64, 8),
                                           (helm.PREC_MIXED, 8)])
def test_unreachable_tolerance_eager_and_captured(prec, max_iter):
    """tol = 1e-30: the loop ends at max_iter or when a step fails to halve
    the residual; HELM_ENOCONV, eagerly and on the captured repeats, with the
    same report and bit-identical last iterates."""
    f, fd = _data(81)
    ud = torch.empty_like(fd)
    with helm.Plan(GRID, inputs.spacing(GRID), OMEGA, precision=prec, tol=1e-30, max_iter=max_iter,
                   check=True) as plan:
        rc = plan.solve(fd, ud, raise_on_error=False)
        rep = plan.report()
        _say("eager", rep)
        assert rc == helm.HELM_ENOCONV and rep["status"] == helm.HELM_ENOCONV
        assert 1 <= rep["iterations"] <= max_iter
        if rep["iterations"] < max_iter:
            assert rep["rel_residual_max"] < 1e-12  # stopped on stagnation at the rounding floor
        u0 = ud.clone()
        res = _oracle_res(u0.cpu().numpy(), f)
        assert np.all(np.isfinite(res)) and np.max(res) <= 1e-10
        assert abs(np.max(res) - rep["rel_residual_max"]) <= 0.5 * np.max(res) + 2e-15
        for k in range(3):  # the second call captures, the third launches the graph
            ud.zero_()
            rc2 = plan.solve(fd, ud, raise_on_error=False)
            rep2 = plan.report()
            torch.cuda.synchronize()
            _say("repeat", k, rep2)
            assert rc2 == helm.HELM_ENOCONV and rep2["status"] == helm.HELM_ENOCONV
            assert rep2["iterations"] == rep["iterations"]
            assert rep2["rel_residual_max"] == rep["rel_residual_max"]
            assert torch.equal(ud, u0)


def test_zero_refinement_steps_reports_enoconv():
    """max_iter = 0 with a tolerance below the first solve's residual: one
    plain solve, HELM_ENOCONV, and the first residual in the report."""
    f, fd = _data(83)
    ud = torch.empty_like(fd)
    with helm.Plan(GRID, inputs.spacing(GRID), OMEGA, precision=helm.PREC_MIXED, tol=1e-10, max_iter=0) as plan:
        rc = plan.solve(fd, ud, raise_on_error=False)
        rep = plan.report()
        _say(rep)
        assert rc == helm.HELM_ENOCONV and rep["iterations"] == 0
        assert rep["rel_residual_first"] == rep["rel_residual_max"] > 1e-10
        res = _oracle_res(ud.cpu().numpy(), f)
        assert abs(np.max(res) - rep["rel_residual_max"]) <= 0.05 * np.max(res)


def test_batch_reports_enoconv_for_one_problem():
    """In a batch graph, the problem whose tolerance cannot be met reports
    HELM_ENOCONV with its last iterate; the other converges."""
    f0, fd0 = _data(85)
    f1, fd1 = _data(87)
    plans = [helm.Plan(GRID, inputs.spacing(GRID), OMEGA, precision=helm.PREC_MIXED),
             helm.Plan(GRID, inputs.spacing(GRID), OMEGA, precision=helm.PREC_MIXED, tol=1e-30, max_iter=3)]
    us = [torch.empty_like(fd0), torch.empty_like(fd1)]
    batch = helm.Batch(plans, max_nrhs=2)
    for _ in range(2):
        batch.solve([fd0, fd1], us)
        r0, r1 = batch.report(0), batch.report(1)
        _say(r0, r1)
        assert r0["status"] == helm.HELM_OK and r0["rel_residual_max"] <= 1e-10
        assert r1["status"] == helm.HELM_ENOCONV and 1 <= r1["iterations"] <= 3
        res1 = _oracle_res(us[1].cpu().numpy(), f1)
        assert np.max(res1) <= 1e-10
        assert abs(np.max(res1) - r1["rel_residual_max"]) <= 0.5 * np.max(res1) + 2e-15
    batch.close()
    for p in plans:
        p.close()
