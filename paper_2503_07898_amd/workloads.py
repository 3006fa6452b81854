"""Seeded synthetic inputs shared by the tests, the oracle runs and bench.py.

This module holds no arithmetic of the method: it only produces initial
macroscopic fields (rho, u) and voxel geometries (fluid masks, level maps).
The method itself (equilibrium, collision, streaming, boundary rules) lives in
the GPU library and, independently, in the oracle.

All arrays are shaped (nz, ny, nx[, 3]) with x fastest in memory, matching the
voxel order x + nx*(y + ny*z) of the library's descriptor.
"""
from __future__ import annotations

import math

import numpy as np


def _grid(nx: int, ny: int, nz: int):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64),
                          np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def taylor_green_2d(n: int, u0: float = 0.05, k: float | None = None):
    """Two-dimensional Taylor-Green vortex extruded along z on an n^3 box.

    u_x = -u0 cos(kx) sin(ky), u_y = u0 sin(kx) cos(ky), u_z = 0,
    rho = 1 - (3 u0^2 / 4) (cos 2kx + cos 2ky)  (pressure p = rho c_s^2 - const).
    Nodes sit at integer coordinates; k defaults to 2 pi / n.
    """
    if k is None:
        k = 2.0 * math.pi / n
    x, y, _ = _grid(n, n, n)
    u = np.zeros((n, n, n, 3))
    u[..., 0] = -u0 * np.cos(k * x) * np.sin(k * y)
    u[..., 1] = u0 * np.sin(k * x) * np.cos(k * y)
    rho = 1.0 - 0.75 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    return rho, u


def taylor_green_3d(n: int, u0: float = 0.05, k: float | None = None):
    """Three-dimensional Taylor-Green vortex (the Re = 1600 benchmark shape).

    u_x = u0 sin(kx) cos(ky) cos(kz), u_y = -u0 cos(kx) sin(ky) cos(kz), u_z = 0,
    p = (u0^2 / 16)(cos 2kx + cos 2ky)(cos 2kz + 2), rho = 1 + 3 p.
    """
    if k is None:
        k = 2.0 * math.pi / n
    x, y, z = _grid(n, n, n)
    u = np.zeros((n, n, n, 3))
    u[..., 0] = u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    u[..., 1] = -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    p = (u0 * u0 / 16.0) * (np.cos(2 * k * x) + np.cos(2 * k * y)) * (np.cos(2 * k * z) + 2.0)
    rho = 1.0 + 3.0 * p
    return rho, u


def tau_for_reynolds(re: float, u0: float, k: float) -> float:
    """tau with Re = u0 / (nu k), nu = (tau - 1/2) / 3."""
    nu = u0 / (re * k)
    return 3.0 * nu + 0.5


def sphere_packing(nx: int, ny: int, nz: int, seed: int = 7898,
                   rmin: float = 8.0, rmax: float = 32.0,
                   target_active: float = 0.30, slab: int = 4,
                   block: int = 4, max_spheres: int = 100000):
    """Obstacle field for the block-sparse wind tunnel.

    Solid = union of spheres with radii ~ U[rmin, rmax] and centres ~ U(box),
    drawn from numpy.random.default_rng(seed).  Spheres that reach into the
    first or last `slab` voxels along x are rejected, so the inflow and outflow
    layers stay fluid.  Spheres are added until the fraction of block^3 blocks
    holding at least one fluid voxel is <= target_active.

    Returns (fluid uint8 (nz,ny,nx), list of (cx, cy, cz, r)).
    """
    assert nx % block == 0 and ny % block == 0 and nz % block == 0
    rng = np.random.default_rng(seed)
    solid = np.zeros((nz, ny, nx), bool)
    bz, by, bx = nz // block, ny // block, nx // block
    nblocks = bx * by * bz
    fluid_count = np.full((bz, by, bx), block ** 3, np.int32)
    active = nblocks
    spheres = []
    while active / nblocks > target_active and len(spheres) < max_spheres:
        r = rng.uniform(rmin, rmax)
        cx, cy, cz = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)
        if cx - r < slab or cx + r > nx - slab:
            continue
        spheres.append((cx, cy, cz, r))
        # voxel bounding box of the sphere, widened to whole blocks
        lo = [max(0, int(math.floor(c - r)) // block * block) for c in (cx, cy, cz)]
        hi = [min(n, (int(math.ceil(c + r)) + block) // block * block)
              for c, n in ((cx, nx), (cy, ny), (cz, nz))]
        zs = np.arange(lo[2], hi[2], dtype=np.float64)[:, None, None]
        ys = np.arange(lo[1], hi[1], dtype=np.float64)[None, :, None]
        xs = np.arange(lo[0], hi[0], dtype=np.float64)[None, None, :]
        inside = (xs - cx) ** 2 + (ys - cy) ** 2 + (zs - cz) ** 2 <= r * r
        sub = solid[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        sub |= inside
        fl = (~sub).reshape((hi[2] - lo[2]) // block, block, (hi[1] - lo[1]) // block, block,
                            (hi[0] - lo[0]) // block, block).sum(axis=(1, 3, 5))
        blk = fluid_count[lo[2] // block:hi[2] // block, lo[1] // block:hi[1] // block,
                          lo[0] // block:hi[0] // block]
        active -= int(np.count_nonzero(blk)) - int(np.count_nonzero(fl))
        blk[...] = fl
    return (~solid).astype(np.uint8), spheres


def random_mask(nx: int, ny: int, nz: int, seed: int, solid_fraction: float = 0.3,
                block: int = 4, empty_block_fraction: float = 0.2):
    """Random block-sparse fluid mask for map and parity tests: some blocks are
    empty, the rest get independent random solid voxels."""
    rng = np.random.default_rng(seed)
    fluid = (rng.random((nz, ny, nx)) >= solid_fraction).astype(np.uint8)
    bz, by, bx = nz // block, ny // block, nx // block
    empty = rng.random((bz, by, bx)) < empty_block_fraction
    e = np.repeat(np.repeat(np.repeat(empty, block, 0), block, 1), block, 2)
    fluid[e] = 0
    return fluid
