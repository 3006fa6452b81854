"""CPU tests of the C ABI and of the host grid builder (no GPU needed).

* liblbm.so loads and exports every function include/lbm.h declares;
* argument and call-order errors come back as status codes with messages;
* the library's index maps equal the oracle's reference builder bit for bit
  on randomized masks (and the reference builder's neighbour table equals an
  O(n^2) brute-force scan);
* the launch structure matches table dissBlock: the naive arm is one kernel
  over n_b + n_nb blocks, memory grouping launches one kernel per group over
  exactly that group's blocks.
"""
import os
import re

import numpy as np
import pytest

from paper_2503_07898_amd import lbm, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = lbm.lib()
    names = _declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def _desc(**kw):
    d = lbm.GridDesc()
    d.kind = kw.get("kind", lbm.DENSE)
    d.nx, d.ny, d.nz = kw.get("n", (8, 8, 8))
    for a in range(3):
        d.periodic[a] = kw.get("periodic", (1, 1, 1))[a]
    d.num_levels = kw.get("levels", 1)
    d.tau = kw.get("tau", 0.6)
    d.storage = kw.get("storage", lbm.F32)
    d.collision = kw.get("collision", lbm.BGK)
    d.schedule = kw.get("schedule", lbm.DISAGG)
    return d


def test_error_paths():
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_grid_create(_desc(tau=0.5))
    assert e.value.status == -1 and "tau" in str(e.value)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_grid_create(_desc(n=(10, 8, 8)))  # block layout needs multiples of 4
    g = lbm.lbm_grid_create(_desc(periodic=(0, 1, 1)))
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_set_boundary(g, lbm.YMIN, lbm.BC_BOUNCE_BACK)  # periodic axis
    assert "periodic" in str(e.value)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_step(g, 1, stream=0)  # before commit/bind/init
    assert e.value.status == -4
    lbm.lbm_grid_commit(g)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_set_boundary(g, lbm.XMIN, lbm.BC_BOUNCE_BACK)  # after commit
    assert e.value.status == -4
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_check(g, stream=0)  # no populations yet
    assert e.value.status == -4
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_grid_bind(g, 0x1000 + 7, 1 << 30, stream=0)  # misaligned workspace
    assert "aligned" in str(e.value)
    lbm.lbm_grid_destroy(g)
    # a voxel on two regularized faces is rejected at commit
    g = lbm.lbm_grid_create(_desc(periodic=(0, 0, 1)))
    lbm.lbm_set_boundary(g, lbm.XMIN, lbm.BC_REG_VELOCITY, (0.05, 0, 0))
    lbm.lbm_set_boundary(g, lbm.YMIN, lbm.BC_REG_PRESSURE, (1, 0, 0))
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_grid_commit(g)
    assert "two regularized" in str(e.value)
    lbm.lbm_grid_destroy(g)
    # dense grids must be all fluid
    fl = np.ones((8, 8, 8), np.uint8)
    fl[3, 3, 3] = 0
    d = _desc()
    d.fluid_mask = fl.ctypes.data
    with pytest.raises(lbm.LbmError):
        lbm.lbm_grid_create(d)


def test_size_limits_and_empty_grids():
    """Block coordinates are packed in 10 bits per axis: 4092 voxels per axis
    is the largest block grid, 4096 is rejected.  A block-sparse grid with no
    fluid voxel and a box with a zero extent are rejected; the dense
    lexicographic arm takes any box size (partial tiles)."""
    g = lbm.lbm_grid_create(_desc(n=(4092, 4, 4)))
    lbm.lbm_grid_commit(g)
    lbm.lbm_grid_destroy(g)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_grid_commit(lbm.lbm_grid_create(_desc(n=(4096, 4, 4))))
    assert "4092" in str(e.value)
    d = _desc(kind=lbm.BLOCK_SPARSE)
    empty = np.zeros((8, 8, 8), np.uint8)
    d.fluid_mask = empty.ctypes.data
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_grid_commit(lbm.lbm_grid_create(d))
    assert "no fluid voxel" in str(e.value)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_grid_commit(lbm.lbm_grid_create(_desc(n=(0, 8, 8), schedule=lbm.PLAIN_SINGLE_KERNEL)))
    for n in ((10, 8, 8), (1, 16, 1), (3, 3, 3)):
        g = lbm.lbm_grid_create(_desc(n=n, schedule=lbm.PLAIN_SINGLE_KERNEL))
        lbm.lbm_grid_commit(g)
        lbm.lbm_grid_destroy(g)


CASES = [
    # (n, periodic, face kinds for XMIN..ZMAX, dense)
    ((16, 12, 8), (False, True, True), ("vel", "pres", "bb", "bb", "bb", "bb"), False),
    ((12, 16, 12), (False, False, False), ("vel", "pres", "bb", "bb", "bb", "bb"), False),
    ((16, 16, 16), (True, True, True), ("bb",) * 6, False),
    ((12, 12, 16), (True, False, False), ("bb", "bb", "bb", "moving", "bb", "bb"), False),
    ((16, 8, 12), (False, False, False), ("bb", "bb", "bb", "bb", "bb", "moving"), True),
    ((8, 12, 16), (True, False, True), ("bb",) * 6, True),
]
KIND = {"bb": lbm.BC_BOUNCE_BACK, "moving": lbm.BC_MOVING_WALL,
        "vel": lbm.BC_REG_VELOCITY, "pres": lbm.BC_REG_PRESSURE}


def _faces(periodic, kinds):
    val = {"bb": (0, 0, 0), "moving": (0.1, 0, 0), "vel": (0.05, 0, 0), "pres": (1.0, 0, 0)}
    return {f: (KIND[kinds[f]], val[kinds[f]]) for f in range(6) if not periodic[f // 2]}


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_index_maps_bit_exact(orc, case, seed):
    n, periodic, kinds, dense = CASES[case]
    if dense:
        fluid = None
    else:
        fluid = workloads.random_mask(*n, seed=seed + 10 * case, solid_fraction=0.15,
                                      empty_block_fraction=0.25)
        if seed == 3:  # some blocks all fluid with full neighbourhoods
            fluid[:, :, :] = 1
            fluid[:4, :4, :4] = 0
    g = lbm.Grid(*n, kind=lbm.DENSE if dense else lbm.BLOCK_SPARSE, periodic=periodic,
                 fluid=fluid, faces=_faces(periodic, kinds), device="cpu")
    okinds = [{"bb": orc.BB, "moving": orc.MOVING, "vel": orc.REG_VEL, "pres": orc.REG_PRES}[k]
              for k in kinds]
    ref = orc.build_block_maps(*n, periodic, fluid, okinds, dense)
    groups = g.index_map(lbm.MAP_GROUPS)
    assert groups[0] == 0  # no resolution jumps on a single-level grid
    assert tuple(groups[1:4]) == ref["groups"]
    nb = int(groups[4])
    assert np.array_equal(g.index_map(lbm.MAP_COORDS).reshape(nb, 3), ref["coords"])
    assert np.array_equal(g.index_map(lbm.MAP_NEIGHBOURS).reshape(nb, 18), ref["nbr"])
    assert np.array_equal(g.index_map(lbm.MAP_FLUIDMASK), ref["fmask"])
    assert np.array_equal(g.index_map(lbm.MAP_CANONICAL), ref["canon"])
    assert g.n == ref["n_fluid"]
    g.close()


@pytest.mark.parametrize("seed", range(6))
def test_reference_builder_neighbours_brute_force(orc, seed):
    n = (12, 8, 16)
    periodic = (seed % 2 == 0, True, seed % 3 == 0)
    fluid = workloads.random_mask(*n, seed=100 + seed, empty_block_fraction=0.3)
    ref = orc.build_block_maps(*n, periodic, fluid, [orc.BB] * 6, False)
    bf = orc.brute_force_neighbours(ref["coords"], periodic, (n[0] // 4, n[1] // 4, n[2] // 4))
    assert np.array_equal(bf, ref["nbr"])
    # Morton order within each group, boundary group first
    keys = [orc.morton_key(*c) for c in ref["coords"]]
    a, b, _ = ref["groups"]
    for lo, hi in ((0, a), (a, a + b), (a + b, len(keys))):
        assert keys[lo:hi] == sorted(keys[lo:hi])


def test_launch_structure_table_dissBlock():
    n = (32, 16, 16)
    fluid, _ = workloads.sphere_packing(*n, seed=5, rmin=2, rmax=5, target_active=0.7)
    faces = {lbm.XMIN: (lbm.BC_REG_VELOCITY, (0.05, 0, 0)), lbm.XMAX: (lbm.BC_REG_PRESSURE, (1, 0, 0)),
             lbm.YMIN: (lbm.BC_BOUNCE_BACK, (0, 0, 0)), lbm.YMAX: (lbm.BC_BOUNCE_BACK, (0, 0, 0)),
             lbm.ZMIN: (lbm.BC_BOUNCE_BACK, (0, 0, 0)), lbm.ZMAX: (lbm.BC_BOUNCE_BACK, (0, 0, 0))}
    common = dict(kind=lbm.BLOCK_SPARSE, periodic=(False, False, False), fluid=fluid, faces=faces,
                  device="cpu")
    naive = lbm.Grid(*n, schedule=lbm.PLAIN_SINGLE_KERNEL, **common)
    disagg = lbm.Grid(*n, schedule=lbm.DISAGG, **common)
    _, gb, gm, gf, total = disagg.index_map(lbm.MAP_GROUPS)
    assert naive.launches() == [total]
    assert sorted(disagg.launches()) == sorted(x for x in (gb, gm, gf) if x > 0)
    assert gb == 2 * (n[1] // 4) * (n[2] // 4)  # inlet and outlet block layers
    # memory grouping needs no boundary metadata: the two arms have the same workspace
    assert naive.workspace_bytes == disagg.workspace_bytes


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("seed", [0, 1])
def test_bitmask_layout_maps(orc, case, seed):
    """Bitmask-based grouping: one Morton order over all blocks, the boundary
    bit of every block equal to the reference builder's classification, and
    one indirect record per fluid voxel of a boundary block on a moving-wall
    or regularized face, numbered in slot order."""
    n, periodic, kinds, dense = CASES[case]
    fluid = None if dense else workloads.random_mask(*n, seed=seed + 10 * case, solid_fraction=0.15,
                                                     empty_block_fraction=0.25)
    g = lbm.Grid(*n, kind=lbm.DENSE if dense else lbm.BLOCK_SPARSE, periodic=periodic, fluid=fluid,
                 faces=_faces(periodic, kinds), schedule=lbm.DISAGG_BITMASK, device="cpu")
    okinds = [{"bb": orc.BB, "moving": orc.MOVING, "vel": orc.REG_VEL, "pres": orc.REG_PRES}[k]
              for k in kinds]
    ref = orc.build_block_maps(*n, periodic, fluid, okinds, dense, grouped=False)
    nb = int(g.index_map(lbm.MAP_GROUPS)[4])
    coords = g.index_map(lbm.MAP_COORDS).reshape(nb, 3)
    assert np.array_equal(coords, ref["coords"])
    keys = [orc.morton_key(*c) for c in coords]
    assert keys == sorted(keys)
    assert np.array_equal(g.index_map(lbm.MAP_NEIGHBOURS).reshape(nb, 18), ref["nbr"])
    assert np.array_equal(g.index_map(lbm.MAP_CANONICAL), ref["canon"])
    bits = g.index_map(lbm.MAP_BOUNDARY_BITS)
    is_b = np.array([(int(bits[b >> 5]) >> (b & 31)) & 1 for b in range(nb)], bool)
    assert np.array_equal(is_b, ref["group"] == 0)
    ids = g.index_map(lbm.MAP_RECORD_IDS)
    fmask = g.index_map(lbm.MAP_FLUIDMASK)
    want, nrec = np.full(nb * 64, -1, np.int32), 0
    valued = [f for f in range(6) if not periodic[f // 2] and kinds[f] != "bb"]
    for b in range(nb):
        if not is_b[b]:
            continue
        for l in range(64):
            if not (int(fmask[b]) >> l) & 1:
                continue
            p = (coords[b, 0] * 4 + (l & 3), coords[b, 1] * 4 + ((l >> 2) & 3), coords[b, 2] * 4 + (l >> 4))
            if any(p[f // 2] == (n[f // 2] - 1 if f & 1 else 0) for f in valued):
                want[b * 64 + l] = nrec
                nrec += 1
    assert np.array_equal(ids, want)
    g.close()
    # the memory-grouped layout carries no records
    m = lbm.Grid(*n, kind=lbm.DENSE if dense else lbm.BLOCK_SPARSE, periodic=periodic, fluid=fluid,
                 faces=_faces(periodic, kinds), device="cpu")
    assert m.index_map(lbm.MAP_RECORD_IDS).size == 0
    m.close()


def test_launch_structure_bitmask_grouping():
    """Table dissBlock, bitmask row: two kernels, each over n_b + n_nb blocks,
    and s_i (4 bytes) of indirect index per slot of every block."""
    n = (32, 16, 16)
    fluid, _ = workloads.sphere_packing(*n, seed=5, rmin=2, rmax=5, target_active=0.7)
    faces = {lbm.XMIN: (lbm.BC_REG_VELOCITY, (0.05, 0, 0)), lbm.XMAX: (lbm.BC_REG_PRESSURE, (1, 0, 0))}
    for f in (lbm.YMIN, lbm.YMAX, lbm.ZMIN, lbm.ZMAX):
        faces[f] = (lbm.BC_BOUNCE_BACK, (0, 0, 0))
    common = dict(kind=lbm.BLOCK_SPARSE, periodic=(False, False, False), fluid=fluid, faces=faces,
                  device="cpu")
    bits = lbm.Grid(*n, schedule=lbm.DISAGG_BITMASK, **common)
    mem = lbm.Grid(*n, schedule=lbm.DISAGG, **common)
    total = int(bits.index_map(lbm.MAP_GROUPS)[4])
    assert bits.launches() == [total, total]
    assert bits.workspace_bytes >= mem.workspace_bytes + 4 * 64 * total
    with pytest.raises(lbm.LbmError):
        lbm.Grid(*n, schedule=lbm.DISAGG_BITMASK, kind=lbm.MULTIRES, levels=2,
                 level_map=np.zeros(n[::-1], np.uint8), device="cpu")


def test_multires_merged_level_updates():
    """A multires level with at most the merge limit of blocks runs each of
    its updates as one launch over all its blocks (2^(L-1-l) updates of
    level l per coarse step).  With every group fused, a coarse level's
    update and the finer level's next update share no buffer one writes and
    the other uses, so they pair into one launch: the 7 level updates of a
    3-level coarse step (levels 0, 1, 0, 2, 0, 1, 0) run as 4 launches
    (0 | 1+0 | 2+0 | 1+0).  The other schedules keep one launch per update.
    Limit 0 gives one launch per non-empty group; a negative limit is
    rejected."""
    n, levels = 64, 3
    lm = workloads.multires_cavity(n)
    faces = {f: (lbm.BC_BOUNCE_BACK, (0, 0, 0)) for f in range(6)}
    faces[lbm.ZMAX] = (lbm.BC_MOVING_WALL, (0.1, 0.0, 0.0))
    g = lbm.Grid(n, n, n, kind=lbm.MULTIRES, levels=levels, level_map=lm, periodic=(False,) * 3,
                 faces=faces, device="cpu")
    groups = [g.index_map(lbm.MAP_GROUPS, level=l) for l in range(levels)]
    totals = [int(x[4]) for x in groups]
    assert max(totals) <= 8192
    merged = g.launches()
    t0, t1, t2 = totals
    assert merged == [t0, t1 + t0, t2 + t0, t1 + t0]
    for sch in (lbm.DISAGG_UNIFORM_FUSED, lbm.PLAIN_SINGLE_KERNEL):
        gs = lbm.Grid(n, n, n, kind=lbm.MULTIRES, levels=levels, level_map=lm, periodic=(False,) * 3,
                      faces=faces, schedule=sch, device="cpu")
        ls = gs.launches()
        assert len(ls) >= 7 and t1 + t0 not in ls and t2 + t0 not in ls, (sch, ls)
        gs.close()
    g.set_merge_limit(0)
    separate = g.launches()
    per_level = [[int(c) for c in x[:4] if c > 0] for x in groups]
    assert sorted(separate) == sorted(c for l, cs in enumerate(per_level) for _ in range(2 ** (levels - 1 - l))
                                      for c in cs)
    assert len(merged) < len(separate)
    with pytest.raises(lbm.LbmError):
        g.set_merge_limit(-1)
    g.close()


def test_xcd_order_covers_every_block_once():
    """The block kernels' workgroup order: logical workgroup
    ((i / C) * 8 + k % 8) * C + i % C for hardware workgroup k (i = k / 8,
    chunks of C = 16), over a grid padded to whole rounds of 8 C; restated
    here, it must reach every logical workgroup exactly once and send the
    padding past the end, for any block count."""
    C = 16

    def remap(k):
        x, i = k & 7, k >> 3
        return ((i // C) * 8 + x) * C + i % C

    for nblocks in (1, 3, 4, 5, 63, 64, 255, 256, 257, 1000, 2474, 23816, 70115):
        nwg = (nblocks + 3) // 4
        grid = (nwg + 8 * C - 1) // (8 * C) * (8 * C)
        v = np.array([remap(k) for k in range(grid)])
        assert sorted(v) == list(range(grid))
        assert np.array_equal(np.sort(v[v < nwg]), np.arange(nwg))
        # hardware workgroup k runs on XCD k % 8: a chunk of C logical
        # workgroups stays on one XCD
        xcd = np.empty(grid, int)
        xcd[v] = np.arange(grid) % 8
        assert np.all(xcd.reshape(-1, C) == xcd.reshape(-1, C)[:, :1])


def test_residency_setting_range():
    """lbm_set_residency takes LBM_RESIDENCY_AUTO (-1), 0 (no cap) or 1..8
    workgroups per CU, in any grid state, and rejects everything else."""
    g = lbm.Grid(16, 16, 16, device="cpu")
    for w in (lbm.RESIDENCY_AUTO, 0, 1, 5, 8):
        g.set_residency(w)
    for w in (-2, 9, 64):
        with pytest.raises(lbm.LbmError):
            g.set_residency(w)
    g.close()


def test_wide_addressing_setting():
    """lbm_set_wide_addressing takes 0 or 1 in any grid state and rejects
    everything else."""
    g = lbm.Grid(16, 16, 16, device="cpu")
    g.set_wide_addressing(True)
    g.set_wide_addressing(False)
    for w in (-1, 2):
        with pytest.raises(lbm.LbmError):
            lbm.lbm_set_wide_addressing(g.h, w)
    g.close()


@pytest.mark.parametrize("case", [0, 1, 4])
@pytest.mark.parametrize("grouped", [True, False])
def test_index_maps_d3q27(orc, case, grouped):
    """D3Q27 layouts: 26 neighbour blocks per block (corners included), maps
    equal to the reference builder's for the same lattice."""
    n, periodic, kinds, dense = CASES[case]
    fluid = None if dense else workloads.random_mask(*n, seed=40 + case, solid_fraction=0.15,
                                                     empty_block_fraction=0.25)
    g = lbm.Grid(*n, kind=lbm.DENSE if dense else lbm.BLOCK_SPARSE, periodic=periodic, fluid=fluid,
                 faces=_faces(periodic, kinds), q=27, device="cpu",
                 schedule=lbm.DISAGG if grouped else lbm.DISAGG_BITMASK)
    okinds = [{"bb": orc.BB, "moving": orc.MOVING, "vel": orc.REG_VEL, "pres": orc.REG_PRES}[k]
              for k in kinds]
    ref = orc.build_block_maps(*n, periodic, fluid, okinds, dense, grouped=grouped, q=27)
    groups = g.index_map(lbm.MAP_GROUPS)
    assert tuple(groups[1:4]) == ref["groups"]
    nb = int(groups[4])
    assert np.array_equal(g.index_map(lbm.MAP_COORDS).reshape(nb, 3), ref["coords"])
    assert np.array_equal(g.index_map(lbm.MAP_NEIGHBOURS).reshape(nb, 26), ref["nbr"])
    assert np.array_equal(g.index_map(lbm.MAP_CANONICAL), ref["canon"])
    g.close()


def test_d3q27_restrictions():
    with pytest.raises(lbm.LbmError):
        lbm.Grid(32, 32, 32, kind=lbm.MULTIRES, levels=2, level_map=np.zeros((32, 32, 32), np.uint8),
                 q=27, device="cpu")
    with pytest.raises(lbm.LbmError):
        lbm.Grid(8, 8, 8, q=23, device="cpu")


MR_CASES = [
    # (levels, n, periodic, face kinds XMIN..ZMAX, obstacle radius or 0)
    (2, (32, 32, 32), (True, True, True), ("bb",) * 6, 0.0),
    (3, (64, 32, 32), (True, True, True), ("bb",) * 6, 0.0),
    (3, (128, 32, 32), (False, True, True), ("vel", "pres", "bb", "bb", "bb", "bb"), 3.0),
    (2, (48, 48, 48), (False, False, False), ("bb", "bb", "bb", "bb", "bb", "moving"), 0.0),
]


@pytest.mark.parametrize("case", range(len(MR_CASES)))
@pytest.mark.parametrize("seed", [0, 1])
def test_multires_index_maps_bit_exact(orc, case, seed):
    """Every level of a multires grid: groups [jump | boundary | masked |
    full] (jump = blocks holding a voxel at distance 0 from a resolution
    jump), block coordinates in Morton order per group, neighbour tables,
    fluid masks and canonical indices equal to the oracle's coordinate-search
    builder, bit for bit."""
    from test_oracle_multires import blob_level_map
    levels, n, periodic, kinds, obst = MR_CASES[case]
    rng = np.random.default_rng(seed + 7 * case)
    centre = (n[0] / 2 + rng.uniform(-3, 3), n[1] / 2 + rng.uniform(-2, 2), n[2] / 2 + rng.uniform(-2, 2))
    radius = 6.0 if obst else rng.uniform(3.0, 6.0)
    lm = blob_level_map(n, levels, centre, radius, band=6.0 if obst else 4.0, periodic=periodic)
    fluid = None
    if obst:
        z, y, x = np.meshgrid(*(np.arange(k, dtype=float) for k in (n[2], n[1], n[0])), indexing="ij")
        fluid = ((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2 > obst ** 2).astype(np.uint8)
    g = lbm.Grid(*n, kind=lbm.MULTIRES, levels=levels, level_map=lm, fluid=fluid, periodic=periodic,
                 faces=_faces(periodic, kinds), tau=0.55, device="cpu")
    okinds = [{"bb": orc.BB, "moving": orc.MOVING, "vel": orc.REG_VEL, "pres": orc.REG_PRES}[k]
              for k in kinds]
    ref = orc.build_multires_maps(*n, levels, periodic, lm, fluid, okinds)
    for l in range(levels):
        r = ref[l]
        groups = g.index_map(lbm.MAP_GROUPS, level=l)
        assert tuple(int(x) for x in groups[:4]) == r["groups4"], l
        assert r["groups4"][0] > 0  # every level meets a resolution jump
        nb = int(groups[4])
        assert np.array_equal(g.index_map(lbm.MAP_COORDS, level=l).reshape(nb, 3), r["coords"])
        assert np.array_equal(g.index_map(lbm.MAP_NEIGHBOURS, level=l).reshape(nb, 18), r["nbr"])
        assert np.array_equal(g.index_map(lbm.MAP_FLUIDMASK, level=l), r["fmask"])
        assert np.array_equal(g.index_map(lbm.MAP_CANONICAL, level=l), r["canon"])
        assert g.n_level(l) == r["n_fluid"]
    g.close()
