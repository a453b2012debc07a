"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module holds no arithmetic of the solver: it only draws right-hand sides
and names the workloads.  Both the HIP path and the CPU oracle receive the
arrays it produces, so they see identical bytes.

Right-hand sides are discrete load vectors f of the system A u = f (Section 2,
eq. (probA)), C-ordered [nrhs][n_1][n_2]([n_3]) with x_1 slowest, complex128.
The paper draws no random numbers; its own experiments use a deterministic
load (0.01 on the first n_1 entries, 1 elsewhere, Section 6), available here
as ``paper_rhs``.  The workloads below use Gaussian loads instead, so that
every eigenmode is excited.
"""

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def omega_for_ppw(n, ppw):
    """Wavenumber giving ``ppw`` mesh points per wavelength on the unit
    interval with n nodes (h = 1/(n-1)): omega = 2*pi/(ppw*h)."""
    return TWO_PI * (n - 1) / ppw


def rhs_seed(config, problem, rhs):
    """Seed of one right-hand side: 1000*config + 10*problem + rhs."""
    return 1000 * config + 10 * problem + rhs


def gaussian(grid, seed):
    """One complex load vector with Re, Im i.i.d. N(0,1) (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(grid))
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return (re + 1j * im).reshape(tuple(grid))


def gaussian_batch(grid, seeds):
    """[len(seeds)][grid] complex128, one seed per right-hand side."""
    return np.stack([gaussian(grid, s) for s in seeds])


def gaussian_device(grid, seeds, device):
    """Same distribution drawn on a device with torch's seeded generator (one
    generator per right-hand side, so any single RHS can be redrawn alone).
    Returns a complex128 tensor [len(seeds)][grid]."""
    import torch
    out = torch.empty((len(seeds),) + tuple(grid), dtype=torch.complex128, device=device)
    view = torch.view_as_real(out)
    for i, s in enumerate(seeds):
        g = torch.Generator(device=device)
        g.manual_seed(int(s))
        view[i].normal_(0.0, 1.0, generator=g)
    return out


def point_source(grid):
    """Load of a unit point source at the centre of the unit square/cube:
    f_i = psi_i(centre).  On an odd axis the centre is node (n-1)/2 (weight 1);
    on an even axis it lies midway between nodes n/2-1 and n/2 (weight 1/2
    each).  The tensor product gives 0.25 on four nodes of an even 2D grid."""
    out = np.ones((), dtype=np.complex128)
    for n in grid:
        w = np.zeros(n)
        if n % 2:
            w[(n - 1) // 2] = 1.0
        else:
            w[n // 2 - 1] = 0.5
            w[n // 2] = 0.5
        out = np.multiply.outer(out, w)
    return out


def paper_rhs(grid):
    """The load of the paper's experiments (Section 6): 0.01 on the first n_1
    entries of the C-ordered vector and 1 elsewhere."""
    f = np.ones(int(np.prod(grid)), dtype=np.complex128)
    f[: grid[0]] = 0.01
    return f.reshape(tuple(grid))


# ---------------------------------------------------------------------------
# Named workloads (all faces absorbing, unit square / cube, h_j = 1/(n_j-1))
# ---------------------------------------------------------------------------

ALL_ABC_2D = 0b1111
ALL_ABC_3D = 0b111111


def workload(name):
    """Return a dict describing a named workload."""
    if name == "2d_128_w80":
        return dict(dim=2, grid=(128, 128), omega=80.0, nrhs=1, config=1,
                    rhs="gaussian+point")
    if name == "2d_4096_ppw10":
        return dict(dim=2, grid=(4096, 4096), omega=TWO_PI * 409.5, nrhs=1, config=2,
                    rhs="gaussian")
    if name == "3d_256_ppw10":
        return dict(dim=3, grid=(256, 256, 256), omega=TWO_PI * 25.5, nrhs=1, config=3,
                    rhs="gaussian")
    if name == "3d_512_ppw10_x16":
        return dict(dim=3, grid=(512, 512, 512), omega=TWO_PI * 51.1, nrhs=16, config=5,
                    rhs="gaussian")
    # the largest shapes of the paper's own experiments (Section 6): omega = 2 pi,
    # n = 2^k + 1, its deterministic load
    if name == "paper_2d_2049":
        return dict(dim=2, grid=(2049, 2049), omega=TWO_PI, nrhs=1, config=6, rhs="paper")
    if name == "paper_3d_513":
        return dict(dim=3, grid=(513, 513, 513), omega=TWO_PI, nrhs=1, config=7, rhs="paper")
    # the anisotropic shapes of the paper's Tables 2 and 4 (same omega and load)
    if name in PAPER_ANISOTROPIC:
        grid = PAPER_ANISOTROPIC[name]
        return dict(dim=len(grid), grid=grid, omega=TWO_PI, nrhs=1, config=8, rhs="paper")
    raise KeyError(name)


PAPER_ANISOTROPIC = {
    "paper_2d_65x2049": (65, 2049),
    "paper_2d_2049x65": (2049, 65),
    "paper_3d_9x513x513": (9, 513, 513),
    "paper_3d_513x9x513": (513, 9, 513),
    "paper_3d_513x513x9": (513, 513, 9),
}
PAPER_SHAPED = ("paper_2d_2049", "paper_3d_513") + tuple(PAPER_ANISOTROPIC)


def batched_2d_problems(count=64, seed=4000):
    """The uneven batch: ``count`` square 2D problems with side drawn uniformly
    from {257, 513, 1025, 2049} and 8-20 points per wavelength."""
    rng = np.random.default_rng(seed)
    sides = rng.choice([257, 513, 1025, 2049], size=count)
    ppw = rng.uniform(8.0, 20.0, size=count)
    return [dict(dim=2, grid=(int(n), int(n)), omega=omega_for_ppw(int(n), float(p)),
                 nrhs=4, ppw=float(p)) for n, p in zip(sides, ppw)]


def spacing(grid):
    """h_j = 1/(n_j - 1) on the unit square / cube."""
    return tuple(1.0 / (n - 1) for n in grid)
