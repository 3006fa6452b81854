"""Pins of the multi-resolution FP64 oracle (CPU).

The paper defines explosion and coalescence only in words, so the oracle's
reading is pinned by properties any correct implementation of it must have:
exact mass conservation in periodic boxes (the operators move every
fine-resolution population exactly once), the uniform state as a fixed
point, reduction to the single-level oracle with one level, and the
Taylor-Green decay rate across a refined slab.
"""
import math

import numpy as np
import pytest

from paper_2503_07898_amd import workloads


def blob_level_map(n, levels, centre, radius, band=4.0, periodic=(True, True, True)):
    nx, ny, nz = n
    bz, by, bx = nz // 4, ny // 4, nx // 4
    zc, yc, xc = np.meshgrid(np.arange(bz) * 4 + 1.5, np.arange(by) * 4 + 1.5,
                             np.arange(bx) * 4 + 1.5, indexing="ij")
    d = np.sqrt((xc - centre[0]) ** 2 + (yc - centre[1]) ** 2 + (zc - centre[2]) ** 2)
    desired = np.full((bz, by, bx), levels - 1, np.int16)
    for l in range(levels - 1):
        desired = np.where((d <= radius + band * (l + 1)) & (desired > l), l, desired)
    return workloads.refine_level_map(nx, ny, nz, levels, desired, periodic)


def random_state(g, seed, amp_u=0.03, amp_rho=0.01):
    rng = np.random.default_rng(seed)
    rho, u = [], []
    for l in range(g.levels):
        shp = g.shape(l)
        rho.append(1 + amp_rho * rng.standard_normal(shp))
        u.append(amp_u * rng.standard_normal(shp + (3,)))
    return g.init_equilibrium(rho, u)


@pytest.mark.parametrize("levels,n", [(2, (32, 32, 32)), (3, (64, 32, 32))])
@pytest.mark.parametrize("collision", [0, 1])
def test_multires_mass_exactly_conserved(orc, levels, n, collision):
    lm = blob_level_map(n, levels, (n[0] / 2, n[1] / 2, n[2] / 2), 6.0)
    counts = [int((lm[::1 << l, ::1 << l, ::1 << l] == l).sum()) for l in range(levels)]
    assert all(c > 0 for c in counts), counts
    g = orc.MultiresGrid(*n, levels=levels, level_map=lm, tau_coarsest=0.56, collision=collision)
    f = random_state(g, 3)
    m0 = g.mass(f)
    f = g.run(f, 200)  # 200 coarse steps
    m1 = g.mass(f)
    assert abs(m1 - m0) / m0 < 1e-13, (m0, m1)


def test_multires_mass_with_obstacle(orc):
    n, levels = (64, 32, 32), 3
    lm = blob_level_map(n, levels, (32, 16, 16), 5.0, band=6.0)
    z, y, x = np.meshgrid(*(np.arange(k, dtype=float) for k in (n[2], n[1], n[0])), indexing="ij")
    fluid = ((x - 32) ** 2 + (y - 16) ** 2 + (z - 16) ** 2 > 9.0).astype(np.uint8)
    g = orc.MultiresGrid(*n, levels=levels, level_map=lm, fluid=fluid, tau_coarsest=0.58)
    f = random_state(g, 5)
    f[0][fluid == 0] = 0.0
    m0 = g.mass(f)
    f = g.run(f, 200)  # 200 coarse steps
    assert abs(g.mass(f) - m0) / m0 < 1e-13


def test_multires_uniform_state_fixed_point(orc):
    n, levels = (64, 32, 32), 3
    lm = blob_level_map(n, levels, (32, 16, 16), 6.0)
    g = orc.MultiresGrid(*n, levels=levels, level_map=lm, tau_coarsest=0.53)
    u0 = np.array([0.04, -0.01, 0.02])
    f = g.init_equilibrium([np.full(g.shape(l), 1.02) for l in range(levels)],
                           [np.broadcast_to(u0, g.shape(l) + (3,)) for l in range(levels)])
    out = g.run(f, 4)
    for l in range(levels):
        a = g.active(l)
        assert np.max(np.abs(out[l][a] - f[l][a])) < 1e-15


def test_multires_single_level_is_single_level_oracle(orc):
    n = 16
    rho, u = workloads.taylor_green_2d(n, 0.05)
    g1 = orc.Grid(n, n, n, tau=0.6)
    f = g1.init_equilibrium(rho, u)
    ref = g1.run(f, 9)
    gm = orc.MultiresGrid(n, n, n, levels=1, level_map=np.zeros((n, n, n), np.uint8), tau_coarsest=0.6)
    out = gm.run([f], 9)[0]
    assert np.max(np.abs(out - ref)) < 1e-16


def test_multires_taylor_green_decay_across_refined_slab(orc):
    """2D Taylor-Green vortex (finest wavelength 64 cells) on a periodic box
    whose middle slab is refined: the amplitude decays as exp(-2 nu k^2 t)
    (finest units) within 2 % at every level."""
    n, levels = (64, 64, 16), 2
    nb = (n[2] // 4, n[1] // 4, n[0] // 4)
    desired = np.ones(nb, np.int16)
    desired[:, :, 6:10] = 0  # x in [24, 40) finest
    lm = workloads.refine_level_map(*n, levels, desired, (True, True, True))
    tau1 = 0.56
    g = orc.MultiresGrid(*n, levels=levels, level_map=lm, tau_coarsest=tau1)
    k = 2 * math.pi / 64
    u0 = 0.03
    nu_f = (g.tau(0) - 0.5) / 3.0  # finest-unit viscosity, = 2 nu_coarse
    rho, u = [], []
    for l in range(levels):
        xs = workloads.level_cell_centres(n[0], l)
        ys = workloads.level_cell_centres(n[1], l)
        zs = workloads.level_cell_centres(n[2], l)
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        uu = np.zeros(Z.shape + (3,))
        uu[..., 0] = -u0 * np.cos(k * X) * np.sin(k * Y)
        uu[..., 1] = u0 * np.sin(k * X) * np.cos(k * Y)
        rho.append(1 - 0.75 * u0 * u0 * (np.cos(2 * k * X) + np.cos(2 * k * Y)))
        u.append(uu)
    f = g.init_equilibrium(rho, u)
    steps = 60  # coarse steps = 120 finest steps
    f = g.run(f, steps)
    decay = math.exp(-2 * nu_f * k * k * 2 * steps)
    for l, (r, v) in enumerate(g.macroscopic(f)):
        a = g.active(l)
        amp = np.sum(v[a] * u[l][a]) / np.sum(u[l][a] * u[l][a])
        assert abs(amp / decay - 1) < 0.02, (l, amp, decay)
        err = np.linalg.norm(v[a] - decay * u[l][a]) / np.linalg.norm(decay * u[l][a])
        assert err < 0.05, (l, err)


def test_multires_lid_cavity_mass_exactly_conserved(orc):
    """Closed cavity refined towards the walls, Ladd lid on the finest level:
    with the moving wall winning at edges its corrections cancel in pairs, so
    the multires scheme still conserves sum_l 8^l sum rho exactly."""
    from paper_2503_07898_amd import workloads
    n = 48
    lm = workloads.multires_cavity(n, shells=(8, 8))
    assert [int((lm[::1 << l, ::1 << l, ::1 << l] == l).sum()) > 0 for l in range(3)] == [True] * 3
    bc = [(orc.BB, (0, 0, 0))] * 6
    bc[orc.ZMAX] = (orc.MOVING, (0.1, 0.0, 0.0))
    g = orc.MultiresGrid(n, n, n, levels=3, level_map=lm, periodic=(False,) * 3, bc=bc, tau_coarsest=0.52)
    f = g.init_equilibrium([np.ones(g.shape(l)) for l in range(3)],
                           [np.zeros(g.shape(l) + (3,)) for l in range(3)])
    # pairwise (numpy) sums: a sequential sum of 2M terms alone is off by ~1e-11

    def mass(f):
        return sum(float(np.sum(f[l][g.active(l)])) * 8 ** l for l in range(3))

    m0 = mass(f)
    f = g.run(f, 20)
    assert abs(mass(f) - m0) / m0 < 1e-13
    # the lid drives the flow: momentum along x appears on the finest level
    _, u0 = g.macroscopic(f)[0]
    assert np.max(u0[..., 0]) > 1e-3


# ---------------------------------------------- multires index-map builder ---

def test_multires_jump_voxels_of_a_refined_slab_closed_form(orc):
    """Two levels in a periodic 64x16x16 box, the finest level on the slab
    16 <= x < 32.  Distance-0 voxels: the two fine layers x = 16 and x = 31
    (16 x 16 each) and the two coarse layers next to the slab, coarse x = 7
    and x = 16 (8 x 8 each); jump blocks: fine block columns bx = 4 and 7
    (4 x 4 blocks each), coarse bx = 1 and 4 (2 x 2 each)."""
    n = (64, 16, 16)
    lm = np.ones((16, 16, 64), np.uint8)
    lm[:, :, 16:32] = 0
    (a0, j0), (a1, j1) = orc.multires_level_masks(*n, 2, (True, True, True), lm)
    assert a0.sum() == 16 * 16 * 16 and a1.sum() == 32 * 8 * 8 - 8 * 8 * 8
    want0 = np.zeros_like(j0)
    want0[:, :, [16, 31]] = True
    want1 = np.zeros_like(j1)
    want1[:, :, [7, 16]] = True
    assert np.array_equal(j0, want0) and np.array_equal(j1, want1)
    maps = orc.build_multires_maps(*n, 2, (True, True, True), lm, None, [orc.BB] * 6)
    assert maps[0]["groups4"] == (2 * 4 * 4, 0, 0, 4 * 4 * 4 - 2 * 4 * 4)
    assert maps[1]["groups4"][0] == 2 * 2 * 2
    assert sorted(set(int(c) for c in maps[0]["coords"][:32, 0])) == [4, 7]
    assert sorted(set(int(c) for c in maps[1]["coords"][:8, 0])) == [1, 4]


def _jump_by_shifts(active_levels, lm, l, periodic):
    """Second formulation of distance 0: the level-l territory array shifted
    by each of the 18 face/edge offsets (np.roll; non-periodic axes padded
    with 'same level' so sources outside the box never count)."""
    s = 1 << l
    terr = lm[::s, ::s, ::s].astype(np.int16)
    act = active_levels
    jump = np.zeros(act.shape, bool)
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
            if 1 <= abs(dx) + abs(dy) + abs(dz) <= 2]
    assert len(offs) == 18
    for dx, dy, dz in offs:
        t = terr
        for ax, d in ((2, dx), (1, dy), (0, dz)):
            if d == 0:
                continue
            t = np.roll(t, d, axis=ax)
            if not periodic[2 - ax]:
                idx = [slice(None)] * 3
                idx[ax] = 0 if d > 0 else -1
                t[tuple(idx)] = l
        jump |= act & (t != l)
    return jump


@pytest.mark.parametrize("seed", range(4))
def test_multires_jump_voxels_match_shift_formulation(orc, seed):
    rng = np.random.default_rng(seed)
    levels = 2 + seed % 2
    n = (64, 32, 32) if levels == 3 else (32, 32, 32)
    periodic = (bool(seed & 1), True, seed != 2)
    centre = rng.uniform(8, 24, 3) * np.array(n) / 32
    lm = blob_level_map(n, levels, tuple(centre), rng.uniform(3, 6), periodic=periodic)
    for l, (act, jmp) in enumerate(orc.multires_level_masks(*n, levels, periodic, lm)):
        assert np.array_equal(jmp, _jump_by_shifts(act, lm, l, periodic)), l
        assert (jmp <= act).all()


@pytest.mark.parametrize("seed", range(3))
def test_multires_block_maps_neighbours_brute_force(orc, seed):
    """Per level: the neighbour tables against the O(n^2) scan, Morton order
    inside each of the groups [jump | boundary | masked | full], and the
    jump group equal to the blocks holding a distance-0 voxel."""
    levels, n = 3, (64, 32, 32)
    periodic = (False, True, True)
    rng = np.random.default_rng(50 + seed)
    lm = blob_level_map(n, levels, (rng.uniform(24, 40), 16, 16), 5.0, band=6.0, periodic=periodic)
    faces = [orc.REG_VEL, orc.REG_PRES, orc.BB, orc.BB, orc.BB, orc.BB]
    masks = orc.multires_level_masks(*n, levels, periodic, lm)
    maps = orc.build_multires_maps(*n, levels, periodic, lm, None, faces)
    for l, m in enumerate(maps):
        nb = tuple(k >> (l + 2) for k in n)
        assert np.array_equal(orc.brute_force_neighbours(m["coords"], periodic, nb), m["nbr"])
        keys = [orc.morton_key(*c) for c in m["coords"]]
        lo = 0
        for cnt in m["groups4"]:
            assert keys[lo:lo + cnt] == sorted(keys[lo:lo + cnt])
            lo += cnt
        jmp = masks[l][1]
        holds = [bool(jmp[z * 4:z * 4 + 4, y * 4:y * 4 + 4, x * 4:x * 4 + 4].any()) for x, y, z in m["coords"]]
        nj = m["groups4"][0]
        assert all(holds[:nj]) and not any(holds[nj:])
