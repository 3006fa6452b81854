"""The benchmark workloads as ready-to-step liblbm grids (GPU).

Each builder creates, binds and initializes a grid with the seeded inputs of
`workloads` and returns it; the counts of updates per step are attached as
`updates_per_step`.
"""
from __future__ import annotations

import functools
import math

import numpy as np

from . import lbm, workloads


def cavity(n=256, storage=lbm.F32, schedule=lbm.DISAGG, tau=0.55, uw=0.1, collision=lbm.BGK, q=19):
    """Dense lid-driven cavity n^3 at rest, bounce-back walls, lid z+ moving
    with (uw, 0, 0)."""
    faces = {f: (lbm.BC_BOUNCE_BACK, (0, 0, 0)) for f in range(6)}
    faces[lbm.ZMAX] = (lbm.BC_MOVING_WALL, (uw, 0.0, 0.0))
    g = lbm.Grid(n, n, n, kind=lbm.DENSE, periodic=(False,) * 3, faces=faces, tau=tau, storage=storage,
                 schedule=schedule, collision=collision, q=q).bind()
    N = g.n
    g.init_equilibrium(np.ones(N), np.zeros((3, N)))
    g.updates_per_step = N
    return g


@functools.lru_cache(maxsize=2)
def _packing(n, seed):
    fluid, _ = workloads.channel_packing(*n, seed=seed)
    fluid.setflags(write=False)
    return fluid


def tunnel(storage=lbm.F32, schedule=lbm.DISAGG, tau=0.6, n=(512, 256, 256), collision=lbm.BGK, seed=7898,
           q=19):
    """Block-sparse wind tunnel through seeded channels of overlapping spheres
    (radii 8-32, <= 30% of 4^3 blocks active), velocity inlet 0.05 on x-,
    pressure outlet rho = 1 on x+, bounce-back walls on y and z."""
    fluid = _packing(tuple(n), seed)
    faces = {lbm.XMIN: (lbm.BC_REG_VELOCITY, (0.05, 0.0, 0.0)),
             lbm.XMAX: (lbm.BC_REG_PRESSURE, (1.0, 0.0, 0.0))}
    for f in (lbm.YMIN, lbm.YMAX, lbm.ZMIN, lbm.ZMAX):
        faces[f] = (lbm.BC_BOUNCE_BACK, (0, 0, 0))
    g = lbm.Grid(*n, kind=lbm.BLOCK_SPARSE, periodic=(False,) * 3, fluid=fluid, faces=faces, tau=tau,
                 storage=storage, schedule=schedule, collision=collision, q=q).bind()
    N = g.n
    u = np.zeros((3, N))
    u[0] = 0.05
    g.init_equilibrium(np.ones(N), u)
    g.updates_per_step = N
    return g


def multires_sphere(storage=lbm.F32, schedule=lbm.DISAGG, scale=1, collision=lbm.BGK, tau=0.52):
    """Flow past a sphere, 3 levels, coarsest 128x64x64 (finest 512x256x256)
    times `scale`, sphere radius 16 finest cells at (128, 128, 128), finest
    level within 24 cells of the sphere, level 1 within a further 48;
    regularized inlet and outlet on x, periodic y and z."""
    n = (512 * scale, 256 * scale, 256 * scale)
    lm, fluid = workloads.multires_sphere(*n, levels=3, center=(128.0 * scale,) * 3, radius=16.0 * scale,
                                          bands=(24.0 * scale, 48.0 * scale))
    faces = {lbm.XMIN: (lbm.BC_REG_VELOCITY, (0.05, 0.0, 0.0)),
             lbm.XMAX: (lbm.BC_REG_PRESSURE, (1.0, 0.0, 0.0))}
    g = lbm.Grid(*n, kind=lbm.MULTIRES, levels=3, level_map=lm, fluid=fluid, periodic=(False, True, True),
                 faces=faces, tau=tau, storage=storage, schedule=schedule, collision=collision).bind()
    for l in range(3):
        N = g.n_level(l)
        u = np.zeros((3, N))
        u[0] = 0.05
        g.init_equilibrium(np.ones(N), u, level=l)
    # every level-l voxel updates 2^(L-1-l) times per coarse step
    g.updates_per_step = sum(g.n_level(l) * 2 ** (2 - l) for l in range(3))
    return g


# Refinement shells (finest cells from the walls, per level boundary) that
# reproduce the voxel distributions of table multiResLbm (millions of
# voxels per level, finest first):
#   320^3: 16.0 / 1.21 / 0.11 ("15, 1, 0.1"), 4 levels 16.0 / 1.21 / 0.078 / 0.004 ("15, 1, 0.1, 0.002")
#   480^3: 54.0 / 4.09 / 0.37 ("53, 4, 0.4"), 4 levels 54.0 / 4.09 / 0.31 / 0.008 ("53, 4, 0.3, 0.008")
#   512^3: 77.6 / 4.09 / 0.37 ("77, 4, 0.4"), 4 levels 77.6 / 2.98 / 0.48 / 0.004 ("73, 3, 0.5, 0.003")
TABLE_SHELLS = {(320, 3): (32, 24), (320, 4): (32, 24, 32), (480, 3): (48, 48), (480, 4): (48, 48, 64),
                (512, 3): (64, 48), (512, 4): (64, 32, 96)}


def multires_cavity(n=512, storage=lbm.F32, schedule=lbm.DISAGG, tau=0.52, uw=0.1, collision=lbm.BGK,
                    levels=3, shells=None):
    """Multi-resolution lid-driven cavity: closed n^3 box (finest
    resolution) refined towards the walls, bounce-back walls, lid z+ moving
    with (uw, 0, 0) on the finest level, tau at the coarsest level.  The
    shells default to TABLE_SHELLS for the table's sizes (512^3, 3 levels:
    77.6M / 4.09M / 0.37M voxels), else to (n/8, 3n/32[, 3n/16])."""
    if shells is None:
        shells = TABLE_SHELLS.get((n, levels))
    if shells is None and levels == 4:
        shells = (n // 8, n // 16, 3 * n // 16)
    lm = workloads.multires_cavity(n, levels=levels, shells=shells)
    faces = {f: (lbm.BC_BOUNCE_BACK, (0, 0, 0)) for f in range(6)}
    faces[lbm.ZMAX] = (lbm.BC_MOVING_WALL, (uw, 0.0, 0.0))
    g = lbm.Grid(n, n, n, kind=lbm.MULTIRES, levels=levels, level_map=lm, periodic=(False,) * 3,
                 faces=faces, tau=tau, storage=storage, schedule=schedule, collision=collision).bind()
    for l in range(levels):
        N = g.n_level(l)
        g.init_equilibrium(np.ones(N), np.zeros((3, N)), level=l)
    g.updates_per_step = sum(g.n_level(l) * 2 ** (levels - 1 - l) for l in range(levels))
    return g


def taylor_green(n=256, re=1600.0, u0=0.05, storage=lbm.F32, collision=lbm.REGULARIZED):
    """3D Taylor-Green vortex on a periodic n^3 box at Reynolds number re."""
    k = 2 * math.pi / n
    rho, u = workloads.taylor_green_3d(n, u0)
    tau = workloads.tau_for_reynolds(re, u0, k)
    coll = lbm.BGK if collision == lbm.MLP else collision
    g = lbm.Grid(n, n, n, kind=lbm.DENSE, tau=tau, collision=coll, storage=storage).bind()
    g.init_equilibrium(rho.reshape(-1), u.reshape(-1, 3).T.copy())
    g.updates_per_step = g.n
    g.tau = tau
    return g
