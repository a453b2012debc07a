"""The dense variant (diagonalisation with the full absorbing-boundary
eigenvectors on the matrix cores, eq. (A2Dinv)) and the transform autotuner,
through the C ABI, against the CPU oracle: FP64 relative error <= 1e-9,
mixed precision relative residual <= 1e-10 with error <= 1e-8."""

import os
import sys

import numpy as np
import pytest

from oracle import fem
from paper_1809_03808_amd import helm, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _abc_tuple(dim, mask):
    return tuple(((mask >> (2 * j)) & 1 == 1, (mask >> (2 * j + 1)) & 1 == 1) for j in range(dim))


def _solve(grid, omega, mask, f, precision, transform, tune_cache=None):
    h = inputs.spacing(grid)
    _say("case", grid, omega, bin(mask), "prec", precision, "transform", transform, "nrhs", f.shape[0])
    with helm.Plan(grid, h, omega, mask, precision=precision, transform=transform,
                   tune_cache=tune_cache) as plan:
        fd = torch.from_numpy(f).cuda()
        ud = torch.empty_like(fd)
        rc = plan.solve(fd, ud, raise_on_error=False)
        torch.cuda.synchronize()
        rep = plan.report()
        u = ud.cpu().numpy()
    return rc, rep, u, h


CASES = [
    ((16, 13), 10.0, 0b1111),
    ((33, 20), 15.0, 0b1111),
    ((64, 100), 40.0, 0b1111),
    ((100, 31), 30.0, 0b1100),   # x1 both Neumann
    ((64, 41), 30.0, 0b0110),    # mixed faces on both axes
    ((257, 65), 80.0, 0b1111),
    ((8, 8, 9), 6.0, 0b111111),
    ((12, 10, 9), 8.0, 0b111111),
    ((16, 8, 13), 12.0, 0b111111),
    ((8, 16, 7), 10.0, 0b110111),
]


@pytest.mark.parametrize("grid,omega,mask", CASES)
def test_dense_fp64_matches_banded_lu(grid, omega, mask):
    f = inputs.gaussian_batch(grid, [71, 72])
    rc, rep, u, h = _solve(grid, omega, mask, f, helm.PREC_FP64, helm.TRANSFORM_DENSE)
    ref = fem.solve(grid, h, omega, _abc_tuple(len(grid), mask), f.reshape(2, -1))
    err = fem.rel_error(u.reshape(2, -1), ref)
    _say("  rel err", err, rep)
    assert rc == helm.HELM_OK and rep["transform"] == helm.TRANSFORM_DENSE
    assert np.max(err) <= 1e-9


@pytest.mark.parametrize("grid,omega", [((64, 77), 35.0), ((12, 20, 9), 12.0), ((257, 33), 90.0)])
def test_dense_mixed_refines_to_1e10(grid, omega):
    mask = (1 << (2 * len(grid))) - 1
    f = inputs.gaussian_batch(grid, [81, 82, 83])
    rc, rep, u, h = _solve(grid, omega, mask, f, helm.PREC_MIXED, helm.TRANSFORM_DENSE)
    abc = _abc_tuple(len(grid), mask)
    ref = fem.solve(grid, h, omega, abc, f.reshape(3, -1))
    err = fem.rel_error(u.reshape(3, -1), ref)
    res = fem.rel_residual(grid, h, omega, abc, u.reshape(3, -1), f.reshape(3, -1))
    _say("  mixed dense err", err, "res", res, rep)
    assert rc == helm.HELM_OK
    assert np.max(res) <= 1e-10 and np.max(err) <= 1e-8


def test_autotuner_decides_and_caches(tmp_path):
    path = str(tmp_path / "tune.txt")
    grid, omega = (48, 40), 25.0
    f = inputs.gaussian_batch(grid, [91])
    rc, rep, u, h = _solve(grid, omega, 0b1111, f, helm.PREC_FP64, helm.TRANSFORM_AUTO, path)
    assert rc == helm.HELM_OK and rep["transform"] in (helm.TRANSFORM_FFT, helm.TRANSFORM_DENSE)
    ref = fem.solve(grid, h, omega, _abc_tuple(2, 0b1111), f.reshape(1, -1))
    assert fem.rel_error(u.reshape(1, -1), ref)[0] <= 1e-9
    everything = open(path).read().splitlines()
    _say("  tune cache:", everything)
    # (the chirp-z axis of length 48 adds its own decision line)
    lines = [ln for ln in everything if " transform=" in ln]
    assert len(lines) == 1 and lines[0].startswith("helm-tune dim=2 grid=48x40x1 prec=0 transform=")
    # a second plan of the same shape takes the cached decisions without timing
    rc2, rep2, u2, _ = _solve(grid, 60.0, 0b1111, f, helm.PREC_FP64, helm.TRANSFORM_AUTO, path)
    assert rc2 == helm.HELM_OK and rep2["transform"] == rep["transform"]
    assert len(open(path).read().splitlines()) == len(everything)
    # a forced choice in the cache is honoured
    forced = helm.TRANSFORM_DENSE if rep["transform"] == helm.TRANSFORM_FFT else helm.TRANSFORM_FFT
    with open(path, "a") as fh:
        fh.write(lines[0].split(" transform=")[0] + f" transform={forced} fft_ms=0 dense_ms=0\n")
    rc3, rep3, u3, _ = _solve(grid, omega, 0b1111, f, helm.PREC_FP64, helm.TRANSFORM_AUTO, path)
    assert rc3 == helm.HELM_OK and rep3["transform"] == forced
    assert fem.rel_error(u3.reshape(1, -1), ref)[0] <= 1e-9


def test_batch_of_dense_and_fft_plans():
    probs = [((40, 33), 20.0, helm.TRANSFORM_DENSE), ((40, 33), 20.0, helm.TRANSFORM_FFT),
             ((12, 10, 9), 8.0, helm.TRANSFORM_DENSE)]
    plans, fs, us, hosts = [], [], [], []
    for i, (grid, omega, tf) in enumerate(probs):
        plans.append(helm.Plan(grid, inputs.spacing(grid), omega, precision=helm.PREC_MIXED, transform=tf))
        f = inputs.gaussian_batch(grid, [inputs.rhs_seed(6, i, r) for r in range(2)])
        hosts.append(f)
        fs.append(torch.from_numpy(f).cuda())
        us.append(torch.empty_like(fs[-1]))
    batch = helm.Batch(plans, max_nrhs=2)
    for launch in range(2):
        batch.solve(fs, us)
        for i, (grid, omega, tf) in enumerate(probs):
            rep = batch.report(i)
            u = us[i].cpu().numpy().reshape(2, -1)
            abc = _abc_tuple(len(grid), (1 << (2 * len(grid))) - 1)
            res = fem.rel_residual(grid, inputs.spacing(grid), omega, abc, u, hosts[i].reshape(2, -1))
            _say(f"  launch {launch} problem {i}: res {res} {rep}")
            assert rep["status"] == helm.HELM_OK and rep["transform"] == tf
            assert np.max(res) <= 1e-10
    batch.close()
    for p in plans:
        p.close()


def test_cached_schedule_decisions_are_honoured(tmp_path):
    """Decisions read from the tune cache (3D: boundary tables from one
    right-hand side on, reductions over the outer modes in layout 3; or
    never the tables) are what the plan runs, and the results meet the bar."""
    grid, omega = (12, 10, 9), 8.0
    h = inputs.spacing(grid)
    f = inputs.gaussian_batch(grid, [97, 98])
    ref = fem.solve(grid, h, omega, ((True, True),) * 3, f.reshape(2, -1))
    for prec in (helm.PREC_FP64, helm.PREC_MIXED):
        key = f"dim=3 grid={grid[0]}x{grid[1]}x{grid[2]} prec={prec}"
        for nmin, want in ((1, helm.BOUNDARY_TABLES), (0, helm.BOUNDARY_LINES)):
            cache = tmp_path / f"tune_{prec}_{nmin}.txt"
            cache.write_text(f"helm-tune {key} layout=3 layout2_ms=1 layout3_ms=0.5\n"
                             f"helm-tune {key} boundary cap_min_nb={nmin}\n")
            with helm.Plan(grid, h, omega, precision=prec, check=prec == helm.PREC_MIXED,
                           tune_cache=str(cache)) as plan:
                fd = torch.from_numpy(f).cuda()
                ud = torch.empty_like(fd)
                plan.solve(fd, ud)
                rep = plan.report()
                u = ud.cpu().numpy().reshape(2, -1)
            err = fem.rel_error(u, ref)
            assert rep["boundary"] == want, (prec, nmin, rep)
            assert np.max(err) <= (1e-9 if prec == helm.PREC_FP64 else 1e-8)
            # nothing of these was measured, so nothing of these was appended
            # (the chirp-z axes of lengths 12 and 10 add their own lines)
            assert len([ln for ln in cache.read_text().splitlines() if " chirp" not in ln]) == 2


@pytest.mark.parametrize("prec", [helm.PREC_MIXED, helm.PREC_FP64])
@pytest.mark.parametrize("grid", [(512, 11), (3, 512, 5), (512, 3, 9)])
def test_fft_tile_decision_timed_cached_and_correct(grid, prec, tmp_path):
    """Plans with a 512-point pass time its forms once (the 128 KB tile, the
    64 KB complex64 tile, the streaming pass) and cache the choice; each
    form, forced through the cache, meets the oracle bar (the plain FP64
    solve without refinement)."""
    omega = 2 * np.pi * (max(grid) - 1) / 12
    h = inputs.spacing(grid)
    dim = len(grid)
    abc = ((True, True),) * dim
    f = inputs.gaussian_batch(grid, [91, 92])
    ref = fem.solve(grid, h, omega, abc, f.reshape(2, -1))
    key = f"dim={dim} grid={grid[0]}x{grid[1]}x{grid[2] if dim == 3 else 1} prec={prec}"
    cache = tmp_path / "tune.txt"
    with helm.Plan(grid, h, omega, precision=prec, tune_cache=str(cache)) as plan:
        pass
    lines = [ln for ln in cache.read_text().splitlines() if "fft512=" in ln]
    assert len(lines) == 1 and lines[0].startswith(f"helm-tune {key} fft512="), lines
    assert "stream_ms=" in lines[0]
    mixed = prec == helm.PREC_MIXED
    for choice in ((0, 1, 2) if mixed else (0, 2)):
        forced = tmp_path / f"forced{choice}.txt"
        forced.write_text(f"helm-tune {key} fft512={choice}\n")
        with helm.Plan(grid, h, omega, precision=prec, check=mixed, tune_cache=str(forced)) as plan:
            fd = torch.from_numpy(f).cuda()
            ud = torch.empty_like(fd)
            plan.solve(fd, ud)
            rep = plan.report()
            u = ud.cpu().numpy().reshape(2, -1)
        assert [ln for ln in forced.read_text().splitlines() if "fft512=" in ln] == [f"helm-tune {key} fft512={choice}"]
        err = fem.rel_error(u, ref)
        assert rep["status"] == 0
        if mixed:
            res = fem.rel_residual(grid, h, omega, abc, u, f.reshape(2, -1))
            assert np.max(res) <= 1e-10 and np.max(err) <= 1e-8
        else:
            assert rep["iterations"] == 0 and np.max(err) <= 1e-9
    if not mixed:
        # the 64 KB complex64 tile is no choice for an FP64 plan: a cached
        # "fft512=1" is ignored and the forms are timed again
        forced = tmp_path / "forced_bad.txt"
        forced.write_text(f"helm-tune {key} fft512=1\n")
        with helm.Plan(grid, h, omega, precision=prec, tune_cache=str(forced)) as plan:
            pass
        lines = [ln for ln in forced.read_text().splitlines() if "fft512=" in ln]
        picked = [t for t in lines[-1].split() if t.startswith("fft512=")]
        assert len(lines) == 2 and picked in (["fft512=0"], ["fft512=2"]), lines


@pytest.mark.parametrize("grid,prec", [
    ((257, 33), helm.PREC_FP64), ((513, 17), helm.PREC_MIXED), ((1025, 9), helm.PREC_FP64),
    ((300, 20), helm.PREC_MIXED), ((17, 513, 9), helm.PREC_FP64), ((129, 9, 7), helm.PREC_MIXED),
    ((2049, 5), helm.PREC_FP64),
])
def test_chirp_pass_decision_timed_cached_and_correct(grid, prec, tmp_path):
    """Chirp-z axes: the plan times the multi-pass and the one-pass
    convolution and caches the choice per axis; either form, forced through
    the cache, meets the oracle bar (FP64 error, mixed residual)."""
    omega = 2 * np.pi * (max(grid) - 1) / 10
    h = inputs.spacing(grid)
    dim = len(grid)
    abc = ((True, True),) * dim
    f = inputs.gaussian_batch(grid, [81, 82])
    ref = fem.solve(grid, h, omega, abc, f.reshape(2, -1))
    key = f"dim={dim} grid={grid[0]}x{grid[1]}x{grid[2] if dim == 3 else 1} prec={prec}"
    axes = [j for j in range(dim - 1) if grid[j] & (grid[j] - 1)]
    cache = tmp_path / "tune.txt"
    with helm.Plan(grid, h, omega, precision=prec, tune_cache=str(cache)) as plan:
        pass
    timed = [ln for ln in cache.read_text().splitlines() if " chirp" in ln]
    assert len(timed) == len(axes), timed
    for choice in (0, 1):
        forced = tmp_path / f"forced{choice}.txt"
        forced.write_text("".join(f"helm-tune {key} chirp{j}={choice}\n" for j in axes))
        with helm.Plan(grid, h, omega, precision=prec, tune_cache=str(forced)) as plan:
            fd = torch.from_numpy(f).cuda()
            ud = torch.empty_like(fd)
            plan.solve(fd, ud)
            rep = plan.report()
            u = ud.cpu().numpy().reshape(2, -1)
        # the chirp decisions were read, not timed
        assert len([ln for ln in forced.read_text().splitlines() if " chirp" in ln]) == len(axes)
        assert rep["status"] == 0
        if prec == helm.PREC_FP64:
            assert np.max(fem.rel_error(u, ref)) <= 1e-9
        else:
            assert np.max(fem.rel_residual(grid, h, omega, abc, u, f.reshape(2, -1))) <= 1e-10
            assert np.max(fem.rel_error(u, ref)) <= 1e-8


@pytest.mark.parametrize("prec", [helm.PREC_MIXED, helm.PREC_FP64])
def test_streaming_pass_walks_several_tiles_per_block(prec, tmp_path):
    """The streaming 512-point pass (forced through the cache) on a volume
    whose passes have more tiles than the device has compute units, with a
    ragged last column tile (63 x 73 = 4599 columns: 144 tiles of 32, the
    last of 23; 288 tiles of 16 for the complex128-input pass), so that every
    block walks several tiles: the solution meets the oracle's residual, and
    the plain FP64 solve needs no refinement."""
    grid = (512, 63, 73)
    omega = 2 * np.pi * 6  # at least 10 points per wavelength on every axis
    h = inputs.spacing(grid)
    abc = ((True, True),) * 3
    f = inputs.gaussian_batch(grid, [93, 94])
    key = f"dim=3 grid={grid[0]}x{grid[1]}x{grid[2]} prec={prec}"
    forced = tmp_path / "tune.txt"
    forced.write_text(f"helm-tune {key} fft512=2\n")
    with helm.Plan(grid, h, omega, precision=prec, check=True, tune_cache=str(forced)) as plan:
        fd = torch.from_numpy(f).cuda()
        ud = torch.empty_like(fd)
        plan.solve(fd, ud)
        rep = plan.report()
        u = ud.cpu().numpy().reshape(2, -1)
    res = fem.rel_residual(grid, h, omega, abc, u, f.reshape(2, -1))
    _say("  streaming pass", prec, rep, res)
    assert rep["status"] == 0 and np.max(res) <= 1e-10
    if prec == helm.PREC_FP64:
        assert rep["iterations"] == 0
