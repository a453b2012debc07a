"""helm_solve_static: the solve that allocates nothing (its workspace is the
library's static device array) against helm_solve on the same plans and
inputs, through the C ABI.  Two calls in a row, the second with a smaller
input; the plans' own workspace and captured graphs are unaffected; sizes
beyond the static array are refused before any work is enqueued."""

import sys

import numpy as np
import pytest

from oracle import fem
from paper_1809_03808_amd import helm, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


KEYS = ("status", "iterations", "precision", "nrhs", "rel_residual_max", "rel_residual_first", "transform",
        "boundary")


def _compare(plan, fd, tag):
    ur = torch.empty_like(fd)
    rc_r = plan.solve(fd, ur, raise_on_error=False)
    rep_r = plan.report()
    us = torch.full_like(fd, complex(7.0, -3.0))
    rc_s = plan.solve_static(fd, us, raise_on_error=False)
    torch.cuda.synchronize()
    rep_s = plan.report()
    d = (torch.max(torch.abs(us - ur)) / torch.max(torch.abs(ur))).item()
    _say(f"{tag}: rc {rc_r}/{rc_s} bit-equal {torch.equal(us, ur)} max rel diff {d:.2e}\n  regular {rep_r}\n  static  {rep_s}")
    assert rc_s == rc_r == helm.HELM_OK
    for k in KEYS:
        assert rep_s[k] == rep_r[k], k
    assert d <= 1e-13
    return us


def test_static_matches_regular_two_calls_second_smaller():
    # first call: 2D 300 x 257 (chirp-z along x1, padded lines), FP64 with the
    # residual check, 3 right-hand sides
    g1 = (300, 257)
    f1 = inputs.gaussian_batch(g1, [91, 92, 93])
    fd1 = torch.from_numpy(f1).cuda()
    with helm.Plan(g1, inputs.spacing(g1), 90.0) as p1:
        u1 = _compare(p1, fd1, "300x257 FP64 x3")
    # second call, smaller: 2D 64 x 77 in mixed precision, 1 right-hand side,
    # also against the oracle
    g2 = (64, 77)
    f2 = inputs.gaussian_batch(g2, [94])
    fd2 = torch.from_numpy(f2).cuda()
    with helm.Plan(g2, inputs.spacing(g2), 35.0, precision=helm.PREC_MIXED) as p2:
        u2 = _compare(p2, fd2, "64x77 mixed x1")
    ref = fem.solve(g2, inputs.spacing(g2), 35.0, ((True, True), (True, True)), f2.reshape(1, -1))
    err = fem.rel_error(u2.cpu().numpy().reshape(1, -1), ref)
    assert err[0] <= 1e-8
    del u1


def test_static_3d_plain_and_dense():
    g = (16, 16, 13)
    f = inputs.gaussian_batch(g, [95, 96])
    fd = torch.from_numpy(f).cuda()
    with helm.Plan(g, inputs.spacing(g), 14.0, check=False) as p:
        _compare(p, fd, "16x16x13 FP64 plain x2")
    with helm.Plan(g, inputs.spacing(g), 14.0, transform=helm.TRANSFORM_DENSE) as p:
        _compare(p, fd[:1].contiguous(), "16x16x13 dense FP64 x1")


def test_static_leaves_plan_workspace_and_graph_intact():
    """Regular solves capture a graph; a static solve in between; the next
    regular call launches the graph and still reproduces the first result."""
    g = (128, 65)
    f = inputs.gaussian_batch(g, [97])
    fd = torch.from_numpy(f).cuda()
    with helm.Plan(g, inputs.spacing(g), 50.0) as p:
        u = torch.empty_like(fd)
        p.solve(fd, u)
        u0 = u.clone()
        p.solve(fd, u)  # captures and launches the graph
        us = torch.empty_like(fd)
        assert p.solve_static(fd, us) == helm.HELM_OK
        u.zero_()
        p.solve(fd, u)  # graph launch on the plan's own workspace
        torch.cuda.synchronize()
        assert torch.equal(u, u0)
        assert torch.max(torch.abs(us - u0)).item() <= 1e-13 * torch.max(torch.abs(u0)).item()


def test_static_refuses_oversize_before_any_work():
    """2048 x 2048 FP64 needs three 64 MiB arrays: more than the static array.
    HELM_ENOMEM, and u is not touched."""
    g = (2048, 2048)
    with helm.Plan(g, inputs.spacing(g), inputs.omega_for_ppw(2048, 10.0)) as p:
        fd = torch.ones((1,) + g, dtype=torch.complex128, device="cuda")
        us = torch.full_like(fd, complex(5.0, 1.0))
        rc = p.solve_static(fd, us, raise_on_error=False)
        torch.cuda.synchronize()
        assert rc == helm.HELM_ENOMEM
        assert p.report()["status"] == helm.HELM_ENOMEM
        assert bool(torch.all(us == complex(5.0, 1.0)))
    g3 = (16, 16, 13)
    with helm.Plan(g3, inputs.spacing(g3), 14.0) as p:
        fd = torch.ones((helm.STATIC_MAX_RHS + 1,) + g3, dtype=torch.complex128, device="cuda")
        us = torch.empty_like(fd)
        assert p.solve_static(fd, us, raise_on_error=False) == helm.HELM_ENOMEM
