"""The shapes of the paper's own experiments (Section 6, Tables 1-4):
omega = 2 pi, n = 2^k + 1 nodes per axis, the paper's load (0.01 on the
first n_1 entries of the vector, 1 elsewhere), absorbing faces everywhere.
Every shape is solved on the GPU in FP64 (checked and refined to 1e-10) and
in mixed precision, and compared with the CPU oracle: banded LU where the
band is narrow (the 2D anisotropic shapes), else the dense separation of
variables refined to a backward error at rounding level (the relative
residual of any FP64 solver stalls well above that for this load: banded LU
reaches about 1e-11 on the 1025 x 9 shape); plus the oracle residual over the
whole array."""

import sys
import time

import numpy as np
import pytest

from oracle import fem, sov
from paper_1809_03808_amd import helm, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _reference(grid, h, omega, abc, f):
    n = int(np.prod(grid))
    # banded LU when the narrowest numbering keeps the band small
    bw = fem.bandwidth(tuple(sorted(grid, reverse=True)))
    if n * bw * bw <= 5e10:
        return fem.solve(grid, h, omega, abc, f[None])[0], "banded LU"
    ur, eta, steps = sov.solve_refined(grid, h, omega, abc, f)
    assert eta <= 1e-15, eta
    return ur, f"separation of variables ({steps} refinement steps, backward error {eta:.1e})"


@pytest.mark.parametrize("name", inputs.PAPER_SHAPED)
def test_paper_shape_by_oracle(name):
    wl = inputs.workload(name)
    grid, omega = wl["grid"], wl["omega"]
    h = inputs.spacing(grid)
    abc = ((True, True),) * len(grid)
    f = inputs.paper_rhs(grid)
    fd = torch.from_numpy(f[None]).cuda()
    t0 = time.time()
    ur, how = _reference(grid, h, omega, abc, f.reshape(-1))
    _say(f"{name}: reference by {how} in {time.time() - t0:.1f} s")
    for prec in (helm.PREC_FP64, helm.PREC_MIXED):
        ud = torch.empty_like(fd)
        with helm.Plan(grid, h, omega, precision=prec) as plan:
            rc = plan.solve(fd, ud, raise_on_error=False)
            rep = plan.report()
        u = ud[0].cpu().numpy().reshape(-1)
        res = fem.rel_residual(grid, h, omega, abc, u[None], f.reshape(1, -1))[0]
        err = float(np.linalg.norm(u - ur) / np.linalg.norm(ur))
        _say(f"  prec {prec}: oracle residual {res:.2e}, error {err:.2e}, report {rep}")
        eta = fem.backward_error(grid, h, omega, abc, u[None], f.reshape(1, -1))[0]
        _say(f"    backward error {eta:.2e}")
        assert rc == helm.HELM_OK and rep["rel_residual_max"] <= 1e-10
        assert res <= 1e-10
        assert err <= 1e-6
