#!/usr/bin/env python3
"""Benchmark of the fast direct Helmholtz solver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one complete helm_solve (forward transforms, the three steps,
inverse transforms, the FP64 residual check that certifies
||f - A u|| / ||f|| <= 1e-10 on the device, and the refinement steps that
check asks for) on inputs already resident in HBM.  The default workload is
the largest single-GPU configuration: the 3D trilinear problem on 512^3 nodes
at 10 points per wavelength (omega = 2 pi * 51.1, absorbing boundary on all
six faces) with 16 seeded Gaussian complex right-hand sides in one solve.
`value` is the complex64-storage + FP64-refinement path (unknowns x RHS per
second); the plain FP64 path on the same inputs is reported beside it
("fp64") with the speedup.  Prints one JSON line.

The line also carries
  roofline      -- the kernel with the largest share of the headline path's
                   device time: its algorithmic bytes per launch (the
                   per-unknown transfers the method must make, counted as
                   below) over its HIP-event-timed mean launch duration,
                   against the 8 TB/s HBM peak; `traffic` is the HBM bytes
                   per launch from the committed rocprofv3 counter summary
                   when it was taken on the current kernel source, else null;
  step_roofline -- the same for whole steps of both paths;
  cpu_baseline  -- the CPU oracle on this host's cores, on one right-hand
                   side of the workload: the dense separation-of-variables
                   solve (eqs. (A2Dinv), (A3Dinv)) and the FP64 residual, with
                   the error of the GPU result against that reference;
  extra         -- the 2D 4096^2 and 3D 256^3 workloads, the 64-problem
                   uneven batch and the paper's own shapes (omega = 2 pi, its
                   load; Tables 1-4) (unless --no-extra).

Algorithmic bytes per unknown (N-sized arrays read or written once; element
e = 16 B for complex128 and 8 B for complex64 storage; a transform counts one
read and one write however many passes it takes; z1 and z2 never stored):
  solve     2D: transforms 2 x 2e + line passes 3e;  3D: 4 x 2e + 4e
            (the first read is of complex128 f, the last write of
            complex128 u);
  residual  read u 16 + read f 16 (+ write r, e, when it feeds a step);
  update    read u 16 + write u 16 (fused into the last inverse transform);
so 2D FP64 one solve + check = 144 B, 3D = 224 B; mixed 2D 72 + 120 k + 32,
3D 112 + 160 k + 32 with k refinement steps.
"""

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the paper's "fast solver" column (Section 6, Tables 1-4; MATLAB on an Intel
# i5-6267U laptop), seconds, for the shapes it reports
PAPER_FAST_SOLVER_S = {"paper_2d_2049": 4.58, "paper_3d_513": 672.27, "paper_2d_65x2049": 0.10,
                       "paper_2d_2049x65": 0.12, "paper_3d_9x513x513": 10.95, "paper_3d_513x9x513": 8.00,
                       "paper_3d_513x513x9": 7.01}
METRIC = "solved unknowns/s at rel. residual ≤1e-10, FP32+refine vs FP64; % HBM peak"


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


_H = "paper_1809_03808_amd/csrc/helm_internal.h"
KERNEL_SOURCES = {
    "lines_kernel": ["paper_1809_03808_amd/csrc/lines.hip", _H],
    "fft_pass_kernel<double2>": ["paper_1809_03808_amd/csrc/fft.hip", _H],
    "fft_pass_kernel<float2>": ["paper_1809_03808_amd/csrc/fft.hip", _H],
    "residual_kernel": ["paper_1809_03808_amd/csrc/stencil.hip", _H],
    "dense_kernel": ["paper_1809_03808_amd/csrc/dense.hip", _H],
}


def _traffic(kernel, key):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current source of that kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    with open(path) as fh:
        db = json.load(fh)
    rec = db.get(key, {}).get(kernel)
    if not rec or rec.get("source_hash") != _source_hash(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        return (max([d.get("num_threads", 1) for d in info] or [1]),
                ",".join(sorted({d.get("internal_api", "?") for d in info})))
    except Exception:
        return 1, "unknown"


# ---------------------------------------------------------------------------
# Algorithmic bytes (the accounting of the module docstring)
# ---------------------------------------------------------------------------

def alg_bytes(dim, mixed, k):
    """Per-unknown algorithmic bytes of one step with k refinement steps, split
    by kernel class: {"transform", "lines", "residual", "total"}."""
    e = 8 if mixed else 16
    ntr = 2 if dim == 2 else 4      # transforms per solve
    nln = 3 if dim == 2 else 4      # N-sized line-pass transfers per solve
    solves = 1 + k
    # every transform reads and writes e per unknown, except: the first
    # solve reads complex128 f and writes complex128 u; a refinement solve's
    # last transform reads z (e) and the fused update reads and writes u
    tr = solves * ntr * 2 * e + 2 * (16 - e) + k * (32 - e)
    lines = solves * nln * e
    resid = k * (32 + e) + 32                   # residuals that feed a step write r; the check only reads
    return {"transform": tr, "lines": lines, "residual": resid, "total": tr + lines + resid}


def _paper_formula(dim, mixed, k):
    """The closed forms quoted in the module docstring (cross-check)."""
    if mixed:
        return (72 + 120 * k + 32) if dim == 2 else (112 + 160 * k + 32)
    solve = 112 if dim == 2 else 192
    return solve + k * (48 + solve + 16) + 32


# ---------------------------------------------------------------------------
# One workload: FP64 and mixed legs, per-kernel event timing, rooflines
# ---------------------------------------------------------------------------

def _time_steps(plan, f, u, steps, warmup):
    import torch
    for _ in range(max(2, warmup)):  # the second call captures the solve graph
        plan.solve(f, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(f, u)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return ms, plan.report()


def _kernel_stats(plan, f, u, steps):
    """The same steps again with every launch bracketed by HIP events on the
    solve's stream (eager launches; the events inflate the step, so step times
    come from _time_steps)."""
    import torch
    plan.profile(True)
    plan.kernel_stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(f, u)
    torch.cuda.synchronize()
    ms_ev = (time.perf_counter() - t0) * 1e3 / steps
    stats = plan.kernel_stats(reset=True)
    plan.profile(False)
    return stats, ms_ev


_CLASS = {"lines_kernel": "lines", "residual_kernel": "residual", "fft_pass_kernel<double2>": "transform",
          "fft_pass_kernel<float2>": "transform"}


def _roofline(stats, steps, ms_ev, dim, mixed, k, N, key):
    """Dominant kernel: its class's algorithmic bytes per step spread over its
    launches, over its mean event-timed launch duration."""
    if not stats:
        return None
    kname, ks = max(stats.items(), key=lambda kv: kv[1]["ms"])
    cls = _CLASS.get(kname)
    ab = alg_bytes(dim, mixed, k)
    launches = ks["calls"] / steps
    per_launch_ms = ks["ms"] / ks["calls"]
    if cls == "transform" and kname != ("fft_pass_kernel<float2>" if mixed else "fft_pass_kernel<double2>"):
        cls = None  # the complex128 boundary-plane passes of the mixed path: no N-sized transfers
    if cls is not None:
        # the class's bytes per step over this kernel's launches per step (in
        # 3D FP64 the volume and the boundary-plane passes share the kernel)
        bytes_launch = ab[cls] * N / launches
    else:
        bytes_launch = ks["bytes"] / ks["calls"]
    achieved = bytes_launch / (per_launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _traffic(kname, key),
            "algorithmic_bytes_per_launch": bytes_launch, "launches_per_step": launches,
            "mean_launch_ms": round(per_launch_ms, 4),
            "timing": f"HIP events around every launch on the solve's stream, {steps} steps "
                      f"({ms_ev:.3f} ms/step with the events)"}


def _per_kernel(stats, steps):
    out = {}
    for k, s in sorted(stats.items(), key=lambda kv: -kv[1]["ms"]):
        out[k] = {"ms_per_step": round(s["ms"] / steps, 4), "launches_per_step": s["calls"] / steps}
    return out


def run_workload(name, steps, warmup, profile=True, keep_rhs0=False):
    """FP64 (checked, refined to tol when needed) and mixed legs of one named
    workload on the same inputs."""
    import torch
    from paper_1809_03808_amd import helm, inputs

    wl = inputs.workload(name)
    grid, omega, nrhs = wl["grid"], wl["omega"], wl["nrhs"]
    dim = len(grid)
    h = inputs.spacing(grid)
    mask = (1 << (2 * dim)) - 1
    N = 1
    for n in grid:
        N *= n
    N *= nrhs
    _log(f"workload {name}: grid {grid} omega {omega:.4f} nrhs {nrhs}")
    if wl["rhs"] == "paper":
        f = torch.from_numpy(inputs.paper_rhs(grid)[None]).to("cuda")
    else:
        f = inputs.gaussian_device(grid, [inputs.rhs_seed(wl["config"], 0, r) for r in range(nrhs)], "cuda")
    u = torch.empty_like(f)
    out = {"workload": name, "grid": list(grid), "omega": omega, "nrhs": nrhs, "unknowns_per_step": N}
    legs = {}
    for leg, prec in (("fp64", helm.PREC_FP64), ("mixed", helm.PREC_MIXED)):
        mixed = prec == helm.PREC_MIXED
        t0 = time.perf_counter()
        plan = helm.Plan(grid, h, omega, mask, precision=prec, check=True)
        setup_s = time.perf_counter() - t0
        ms, rep = _time_steps(plan, f, u, steps, warmup)
        k = rep["iterations"]
        val = N / (ms * 1e-3)
        ab = alg_bytes(dim, mixed, k)
        assert ab["total"] == _paper_formula(dim, mixed, k), (ab, _paper_formula(dim, mixed, k))
        step_frac = ab["total"] * N / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
        d = {"ms_per_step": round(ms, 4), "value": val, "unit": "unknowns/s", "status": rep["status"],
             "refinement_steps": k, "rel_residual": rep["rel_residual_max"],
             "rel_residual_first_solve": rep["rel_residual_first"], "setup_s": round(setup_s, 2),
             "step_roofline": {"algorithmic_bytes_per_unknown": ab, "achieved_GBs":
                               round(ab["total"] * N / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                               "frac": round(step_frac, 4)}}
        if profile:
            stats, ms_ev = _kernel_stats(plan, f, u, steps)
            d["roofline"] = _roofline(stats, steps, ms_ev, dim, mixed, k, N, f"{name}/{leg}")
            d["kernels"] = _per_kernel(stats, steps)
            # per class, the fraction of peak by the algorithmic bytes
            cls = {}
            for kn, s in stats.items():
                c = _CLASS.get(kn)
                if c:
                    cls[c] = cls.get(c, 0.0) + s["ms"] / steps
            d["class_frac"] = {c: round(ab[c] * N / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) for c, t in cls.items()}
        _log(f"  {leg}: {ms:.3f} ms/step, {val / 1e9:.3f} G unknowns/s, step frac {step_frac:.3f}, report {rep}")
        if d.get("roofline"):
            _log(f"    roofline {d['roofline']}")
            for kn, s in d["kernels"].items():
                _log(f"    {kn:28s} {s['ms_per_step']:9.3f} ms/step {s['launches_per_step']:5.1f} launches")
        legs[leg] = d
        plan.close()
        if rep["status"] != 0 or rep["rel_residual_max"] > 1e-10:
            _log(f"WARNING: {leg} residual check failed", rep)
    if keep_rhs0:
        out["_f0"] = f[0].cpu().numpy()
        out["_u0"] = u[0].cpu().numpy()  # the mixed leg's result (ran last)
    del f, u
    torch.cuda.empty_cache()
    out["fp64"] = legs["fp64"]
    out["mixed"] = legs["mixed"]
    out["mixed_speedup_vs_fp64"] = round(legs["fp64"]["ms_per_step"] / legs["mixed"]["ms_per_step"], 3)
    return out


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on one right-hand side of the workload
# ---------------------------------------------------------------------------

def cpu_baseline(name, f0, u0):
    """The second CPU oracle (dense separation of variables with the
    absorbing-boundary eigenvectors, one zgtsv per mode) on right-hand side 0
    of the workload, the FP64 residual of its result, and the error of the
    GPU's mixed-path result against it."""
    import numpy as np
    from oracle import fem, sov
    from paper_1809_03808_amd import inputs
    wl = inputs.workload(name)
    grid, omega = wl["grid"], wl["omega"]
    h = inputs.spacing(grid)
    abc = ((True, True),) * len(grid)
    cores, blas = _blas_threads()
    t0 = time.perf_counter()
    eig = [sov.axis_eigenpairs(grid[j], h[j], omega, True, True) for j in range(len(grid) - 1)]
    t_eig = time.perf_counter() - t0
    t0 = time.perf_counter()
    ur = sov.solve(grid, h, omega, abc, f0.reshape(-1), eig=eig)
    t_sov = time.perf_counter() - t0
    t0 = time.perf_counter()
    res_ref = float(fem.rel_residual(grid, h, omega, abc, ur[None], f0.reshape(1, -1))[0])
    t_res = time.perf_counter() - t0
    res_gpu = float(fem.rel_residual(grid, h, omega, abc, u0.reshape(1, -1), f0.reshape(1, -1))[0])
    err = float(np.linalg.norm(u0.reshape(-1) - ur) / np.linalg.norm(ur))
    n = int(np.prod(grid))
    return {"value": n / t_sov, "unit": "unknowns/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": _cpu_model(), "blas": blas, "seconds": round(t_sov, 2),
            "eigen_setup_s": round(t_eig, 2), "fp64_residual_s": round(t_res, 2),
            "fp64_residual_unknowns_per_s": n / t_res,
            "reference_rel_residual": res_ref,
            "gpu_mixed_rel_residual_by_oracle": res_gpu,
            "gpu_mixed_rel_error_vs_oracle": err,
            "sample": f"right-hand side 0 of {name} ({'x'.join(str(g) for g in grid)} nodes): dense separation "
                      "of variables in complex128 (eigenpairs set up beforehand, not timed), then the oracle's "
                      "FP64 matrix-free residual"}


def batch_leg(steps, warmup, count=64):
    """The uneven batch: ``count`` square 2D problems (sides from {257, 513,
    1025, 2049}, 8-20 points per wavelength, 4 Gaussian right-hand sides
    each, complex64 storage + FP64 refinement to 1e-10) solved by one graph
    launch per step.  Also times the same problems solved one after another
    by separate helm_solve calls on one stream (each call synchronises; after
    its first call each plan launches its own captured solve)."""
    import torch
    from paper_1809_03808_amd import helm, inputs
    import tempfile
    probs = inputs.batched_2d_problems(count=count, seed=4000)
    tune = os.path.join(tempfile.mkdtemp(prefix="helm_tune_"), "tune.txt")
    t0 = time.perf_counter()
    plans, fs, us = [], [], []
    for i, pr in enumerate(probs):
        g = pr["grid"]
        plans.append(helm.Plan(g, inputs.spacing(g), pr["omega"], precision=helm.PREC_MIXED,
                               transform=helm.TRANSFORM_AUTO, tune_cache=tune))
        fs.append(inputs.gaussian_device(g, [inputs.rhs_seed(4, i, r) for r in range(pr["nrhs"])], "cuda"))
        us.append(torch.empty_like(fs[-1]))
    setup_s = time.perf_counter() - t0
    unknowns = sum(pr["grid"][0] * pr["grid"][1] * pr["nrhs"] for pr in probs)
    batch = helm.Batch(plans, max_nrhs=4)
    t0 = time.perf_counter()
    batch.solve(fs, us)
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t0
    for _ in range(warmup):
        batch.solve(fs, us)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.solve(fs, us)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    reps = [batch.report(i) for i in range(len(plans))]
    chosen = {}
    for pr, r in zip(probs, reps):
        key = f"{pr['grid'][0]}:{'dense' if r['transform'] == helm.TRANSFORM_DENSE else 'fft'}"
        chosen[key] = chosen.get(key, 0) + 1
    with open(tune) as fh:
        tune_lines = [ln.strip() for ln in fh if ln.strip()]
    for _ in range(2):
        for p, f, u in zip(plans, fs, us):
            p.solve(f, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, f, u in zip(plans, fs, us):
        p.solve(f, u)
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3
    batch.close()
    for p in plans:
        p.close()
    sizes = {}
    for pr in probs:
        sizes[pr["grid"][0]] = sizes.get(pr["grid"][0], 0) + 1
    return {"workload": f"{count} independent 2D problems, sides {dict(sorted(sizes.items()))}, "
                        "8-20 points/wavelength, 4 Gaussian RHS each, complex64 + FP64 refinement to 1e-10, "
                        "one graph launch per step",
            "value": unknowns / (ms * 1e-3), "unit": "unknowns/s", "ms_per_step": round(ms, 4),
            "unknowns_per_step": unknowns, "steps": steps,
            "status_ok": all(r["status"] == 0 for r in reps),
            "rel_residual_max": max(r["rel_residual_max"] for r in reps),
            "refinement_steps_max": max(r["iterations"] for r in reps),
            "sequential_calls_ms": round(seq_ms, 3), "batch_speedup_vs_sequential_calls": round(seq_ms / ms, 3),
            "transform_chosen": chosen, "tuner_decisions": tune_lines,
            "setup_s": round(setup_s, 2), "first_call_s": round(first_s, 2)}


def describe(name):
    from paper_1809_03808_amd import inputs
    wl = inputs.workload(name)
    grid, dim = wl["grid"], len(wl["grid"])
    load = ("seeded Gaussian complex" if wl["rhs"] == "gaussian" else
            "Gaussian complex plus a centre point source" if wl["rhs"] == "gaussian+point" else
            "paper load (0.01 on the first n1 entries, 1 elsewhere)")
    return (f"{name}: {dim}D {'bilinear Q1' if dim == 2 else 'trilinear Q1'} FE Helmholtz "
            f"{'x'.join(str(n) for n in grid)} nodes, unit {'square' if dim == 2 else 'cube'}, "
            f"first-order ABC on all faces, omega={wl['omega']:.6f}, {wl['nrhs']} {load} RHS in one solve")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="3d_512_ppw10_x16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 4096^2, 256^3 and batch legs")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip per-kernel event timing (pure wall-clock run)")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None,
                    help="profiling aid: run one leg of the workload only, no extras, no JSON roofline")
    ap.add_argument("--transform", choices=["fft", "dense"], default="fft",
                    help="with --only: the periodised-axis transform of the plan")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="after the run, copy a buffer of this size (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(independent right-hand sides or problems shard across GPUs without communication).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.workload == "2d_batch64":
        b = batch_leg(args.steps, args.warmup)
        _log("batch", b)
        line = {"metric": METRIC, "value": b["value"], "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": b["ms_per_step"], "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64", "data": "synthetic",
                "config": {"workload": b["workload"]}, "batch": b, "roofline": None, "cpu_baseline": None}
        print(json.dumps(line), flush=True)
        return

    if args.only:
        from paper_1809_03808_amd import helm, inputs
        wl = inputs.workload(args.workload)
        grid = wl["grid"]
        f = inputs.gaussian_device(grid, [inputs.rhs_seed(wl["config"], 0, r) for r in range(wl["nrhs"])], "cuda")
        u = torch.empty_like(f)
        prec = helm.PREC_FP64 if args.only == "fp64" else helm.PREC_MIXED
        tf = helm.TRANSFORM_DENSE if args.transform == "dense" else helm.TRANSFORM_FFT
        plan = helm.Plan(grid, inputs.spacing(grid), wl["omega"], precision=prec, check=True, transform=tf)
        ms, rep = _time_steps(plan, f, u, args.steps, args.warmup)
        _log(f"{args.workload} {args.only}: {ms:.3f} ms/step report {rep}")
        if not args.no_profile:
            stats, _ = _kernel_stats(plan, f, u, args.steps)
            for kn, s in _per_kernel(stats, args.steps).items():
                _log(f"    {kn:28s} {s['ms_per_step']:9.3f} ms/step {s['launches_per_step']:5.1f} launches")
        plan.close()
        if args.copy_calibration_gib > 0:
            nbytes = int(args.copy_calibration_gib * (1 << 30))
            a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
            b = torch.empty_like(a)
            torch.cuda.synchronize()
            b.copy_(a)
            torch.cuda.synchronize()
            _log(f"copy calibration: {nbytes} bytes read, {nbytes} bytes written")
        print(json.dumps({"workload": args.workload, "leg": args.only, "transform": args.transform,
                          "ms_per_step": ms, "report": rep}))
        return

    head = run_workload(args.workload, args.steps, args.warmup, profile=not args.no_profile,
                        keep_rhs0=not args.no_cpu_baseline)
    f0, u0 = head.pop("_f0", None), head.pop("_u0", None)
    extra = {}
    if not args.no_extra:
        for name in ("2d_4096_ppw10", "3d_256_ppw10"):
            if name != args.workload:
                extra[name] = run_workload(name, max(args.steps, 10), args.warmup, profile=not args.no_profile)
        extra["2d_batch64"] = batch_leg(max(3, args.steps // 4), 1)
        _log("batch", extra["2d_batch64"])
        # the paper's own shapes (omega = 2 pi, its load), with its MATLAB
        # fast-solver times on a laptop CPU as context (not a target)
        from paper_1809_03808_amd import inputs
        for name in inputs.PAPER_SHAPED:
            d = run_workload(name, 5, 2, profile=False)
            d["paper_fast_solver_s_laptop_matlab"] = PAPER_FAST_SOLVER_S.get(name)
            extra[name] = d
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, f0, u0)
        _log("cpu baseline", cpu)
    mixed = head["mixed"]
    line = {
        "metric": METRIC,
        "value": mixed["value"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {"workload": describe(args.workload),
                   "path": "complex64 storage and transforms, FP64 line recurrences, FP64 residual and "
                           "update (iterative refinement to rel. residual 1e-10)",
                   "rel_residual": mixed["rel_residual"], "refinement_steps": mixed["refinement_steps"]},
        "roofline": mixed.get("roofline"),
        "step_roofline": {"mixed": mixed["step_roofline"], "fp64": head["fp64"]["step_roofline"]},
        "fp64": head["fp64"],
        "mixed": mixed,
        "mixed_speedup_vs_fp64": head["mixed_speedup_vs_fp64"],
        "extra": extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
