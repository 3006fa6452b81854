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


def channel_packing(nx: int, ny: int, nz: int, seed: int = 7898,
                    rmin: float = 8.0, rmax: float = 32.0,
                    target_active: float = 0.30, block: int = 4):
    """Pore-channel geometry for the block-sparse wind tunnel.

    Fluid = union of spheres strung into channels that cross the box along x.
    A channel draws one radius r ~ U[rmin, rmax] and an entry point
    (y, z) ~ U(inlet face); its sphere centres start on the inlet plane
    x = 0 and advance by r/2 along x, each step moving the centre by
    U[-r/4, r/4] along y and z (clamped to the box), until a sphere reaches
    past the outlet plane.  Channels are drawn from
    numpy.random.default_rng(seed) and kept while the fraction of block^3
    blocks holding at least one fluid voxel stays <= target_active (the
    channel that would exceed it ends the draw).

    Consecutive spheres of a channel overlap by half a radius, so every
    channel joins the inlet to the outlet through openings of at least
    0.97 r, and channels that meet join.

    Returns (fluid uint8 (nz, ny, nx), number of channels).
    """
    assert nx % block == 0 and ny % block == 0 and nz % block == 0
    rng = np.random.default_rng(seed)
    fluid = np.zeros((nz, ny, nx), bool)
    nblocks = (nx // block) * (ny // block) * (nz // block)

    def active(f):
        return f.reshape(nz // block, block, ny // block, block, nx // block, block).any(axis=(1, 3, 5))

    channels = 0
    while True:
        r = rng.uniform(rmin, rmax)
        y, z = rng.uniform(0, ny), rng.uniform(0, nz)
        x = 0.0
        cand = fluid.copy()
        while x - r < nx:
            lo = [max(0, int(math.floor(c - r))) for c in (x, y, z)]
            hi = [min(n, int(math.ceil(c + r)) + 1) for c, n in ((x, nx), (y, ny), (z, nz))]
            zs = np.arange(lo[2], hi[2], dtype=np.float64)[:, None, None]
            ys = np.arange(lo[1], hi[1], dtype=np.float64)[None, :, None]
            xs = np.arange(lo[0], hi[0], dtype=np.float64)[None, None, :]
            cand[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] |= (xs - x) ** 2 + (ys - y) ** 2 + (zs - z) ** 2 <= r * r
            x += r / 2
            y = min(max(y + rng.uniform(-r / 4, r / 4), 0.0), float(ny))
            z = min(max(z + rng.uniform(-r / 4, r / 4), 0.0), float(nz))
        if channels > 0 and np.count_nonzero(active(cand)) > target_active * nblocks:
            break
        fluid = cand
        channels += 1
    return fluid.astype(np.uint8), channels


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


# ------------------------------------------------------ multi-resolution ---

def refine_level_map(nx: int, ny: int, nz: int, levels: int, desired: np.ndarray,
                     periodic=(True, True, True)) -> np.ndarray:
    """Block-aligned, 2:1-balanced level map (uint8 (nz, ny, nx), 0 = finest).

    desired: int array (nz/4, ny/4, nx/4), the coarsest level allowed for each
    finest-level block of 4^3 voxels.  A level-l block covers 2^l finest
    blocks per axis.  Starting from the coarsest level, every block whose
    region asks for a finer level is split into 8; then blocks are split
    until every two blocks that share a face, edge or corner differ by at
    most one level.
    """
    L = levels
    top = 4 << (L - 1)
    assert nx % top == 0 and ny % top == 0 and nz % top == 0, "box must hold whole coarsest blocks"
    shp = (nz // 4, ny // 4, nx // 4)
    des = np.asarray(desired).reshape(shp)
    lv = np.full(shp, L - 1, np.int16)

    def region_reduce(a, s, fn):
        r = a.reshape(shp[0] // s, s, shp[1] // s, s, shp[2] // s, s)
        return fn(fn(fn(r, axis=5), axis=3), axis=1)

    def expand(a, s):
        return np.repeat(np.repeat(np.repeat(a, s, 0), s, 1), s, 2)

    for l in range(L - 1, 0, -1):
        s = 1 << l
        at_l = region_reduce(lv == l, s, np.all)
        need = region_reduce(des, s, np.min) < l
        lv[expand(at_l & need, s)] = l - 1

    def neighbour_min(a):
        # 26-neighbourhood minimum; periodic axes wrap, others repeat the edge
        m = a.copy()
        pad = np.pad(a, 1, mode="wrap")
        for ax in range(3):
            if not periodic[2 - ax]:
                sl = [slice(None)] * 3
                src = [slice(None)] * 3
                sl[ax], src[ax] = slice(0, 1), slice(1, 2)
                pad[tuple(sl)] = pad[tuple(src)]
                sl[ax], src[ax] = slice(-1, None), slice(-2, -1)
                pad[tuple(sl)] = pad[tuple(src)]
        for dz in range(3):
            for dy in range(3):
                for dx in range(3):
                    m = np.minimum(m, pad[dz:dz + shp[0], dy:dy + shp[1], dx:dx + shp[2]])
        return m

    while True:
        nm = neighbour_min(lv)
        bad = lv - nm >= 2
        if not bad.any():
            break
        for l in range(L - 1, 1, -1):
            s = 1 << l
            reg = region_reduce(bad & (lv == l), s, np.any)
            lv[expand(reg, s) & (lv == l)] = l - 1
    return expand(lv.astype(np.uint8), 4)


def multires_sphere(nx: int = 512, ny: int = 256, nz: int = 256, levels: int = 3,
                    center=(128.0, 128.0, 128.0), radius: float = 16.0, bands=(24.0, 48.0),
                    periodic=(False, True, True)):
    """Flow past a sphere on a multi-resolution grid (finest resolution box).

    Finest level (0) on every block within bands[0] finest cells of the
    sphere surface, level 1 within a further bands[1] cells, coarser beyond.
    Returns (level_map uint8 (nz,ny,nx), fluid uint8 (nz,ny,nx)); the solid
    sphere is the set of voxel positions (integer coordinates) with
    |p - center| <= radius.
    """
    bz, by, bx = nz // 4, ny // 4, nx // 4
    zc, yc, xc = np.meshgrid(np.arange(bz) * 4 + 1.5, np.arange(by) * 4 + 1.5,
                             np.arange(bx) * 4 + 1.5, indexing="ij")
    d = np.sqrt((xc - center[0]) ** 2 + (yc - center[1]) ** 2 + (zc - center[2]) ** 2)
    dsurf = np.maximum(np.abs(d - radius) - 2.0 * math.sqrt(3.0), 0.0)
    desired = np.full((bz, by, bx), levels - 1, np.int16)
    lim = 0.0
    for l, b in enumerate(bands[: levels - 1]):
        lim += b
        desired = np.where((dsurf <= lim) & (desired > l), l, desired)
    lm = refine_level_map(nx, ny, nz, levels, desired, periodic)
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    solid = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2 <= radius * radius
    return lm, (~solid).astype(np.uint8)


def multires_cavity(n: int = 512, levels: int = 3, shells=None):
    """Multi-resolution lid-driven cavity (the shape of the paper's multires
    benchmark, table multiResLbm): a closed n^3 box (finest resolution),
    finest level on every block within shells[0] finest cells of a wall,
    level 1 within a further shells[1] cells, coarser inside.

    The default shells (n/8, 3n/32) put 57.8% / 24.4% / 17.8% of the box
    volume on levels 0 / 1 / 2: at n = 512 that is 77.6M, 4.09M and 0.37M
    voxels, the distribution "77, 4, 0.4" of the paper's 512^3 row.
    Returns the level map (uint8 (n, n, n)); every voxel is fluid.
    """
    if shells is None:
        shells = (n // 8, 3 * n // 32)
    nb = n // 4
    c = np.arange(nb)
    # distance (finest cells) from each finest 4^3 block to the nearest wall
    d1 = np.minimum(c, nb - 1 - c) * 4
    d = np.minimum(np.minimum(d1[:, None, None], d1[None, :, None]), d1[None, None, :])
    desired = np.full((nb, nb, nb), levels - 1, np.int16)
    lim = 0
    for l, t in enumerate(shells[: levels - 1]):
        lim += t
        desired = np.where((d < lim) & (desired > l), l, desired)
    return refine_level_map(n, n, n, levels, desired, periodic=(False, False, False))


def level_cell_centres(n: int, l: int) -> np.ndarray:
    """Finest-unit coordinate of the centres of level-l cells along an axis
    of n finest voxels (finest voxel i sits at i)."""
    s = 1 << l
    return np.arange(n >> l, dtype=np.float64) * s + (s - 1) / 2.0


# --------------------------------------------------------- learned closure ---

def mlp_he_uniform(seed: int, sizes=(19, 64, 64, 19)):
    """Initial weights of the closure network: He-uniform
    U(-sqrt(6/fan_in), +sqrt(6/fan_in)) per layer from default_rng(seed), zero
    biases.  Returns [W1, b1, W2, b2, W3, b3] as float64 arrays, W_k shaped
    (fan_in, fan_out)."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = math.sqrt(6.0 / a)
        out.append(rng.uniform(-lim, lim, (a, b)))
        out.append(np.zeros(b))
    return out


def sample_indices(seed: int, n: int, population: int) -> np.ndarray:
    """n indices drawn uniformly with replacement from range(population)."""
    return np.random.default_rng(seed).integers(0, population, n, dtype=np.int64)
