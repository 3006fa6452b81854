"""Degenerate and ragged inputs on the GPU path against the FP64 oracle
(MI355X): boxes whose sizes are not multiples of the 64x4 tile of the
lexicographic kernel, a one-voxel-wide periodic Couette channel, a grid of a
single 4^3 block (every voxel on a wall, the lid on one face), and a sparse
grid of isolated fluid voxels (every pull bounces back).  Bars as in the
other parity tests: 1e-5 relative L2 on velocity for FP32 storage, bit-exact
between arms that share arithmetic, and exact mass conservation up to FP32
rounding where the rules conserve it exactly.
"""
import sys

import numpy as np
import pytest

from paper_2503_07898_amd import lbm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lbm.lib()


def canon(arr, fluid):
    if fluid is None:
        return arr.reshape((-1,) + arr.shape[3:])
    return arr[np.asarray(fluid, bool)]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


KIND = {lbm.BC_BOUNCE_BACK: "BB", lbm.BC_MOVING_WALL: "MOVING", lbm.BC_REG_VELOCITY: "REG_VEL",
        lbm.BC_REG_PRESSURE: "REG_PRES"}


def oracle_run(orc, n, steps, rho, u, fluid, periodic, faces, tau):
    bc = [(orc.BB, (0, 0, 0))] * 6
    for f, (k, v) in faces.items():
        bc[f] = (getattr(orc, KIND[k]), v)
    og = orc.Grid(*n, periodic=periodic, fluid=fluid, bc=bc, tau=tau)
    f = og.run(og.init_equilibrium(rho, u), steps)
    r, v = og.macroscopic(f)
    return canon(r, fluid), canon(v, fluid)


def gpu_run(n, steps, rho, u, fluid, periodic, faces, tau, **kw):
    g = lbm.Grid(*n, fluid=fluid, periodic=periodic, faces=faces, tau=tau, **kw).bind()
    g.init_equilibrium(canon(rho, fluid), canon(u, fluid).T.copy())
    m0 = g.reduce().cpu().numpy()[0]
    g.step(steps)
    r, v = g.macroscopic()
    m1 = g.reduce().cpu().numpy()[0]
    return g, r.cpu().numpy(), v.cpu().numpy().T, m0, m1


@pytest.mark.parametrize("n,periodic", [((20, 12, 7), (True, True, True)), ((70, 5, 9), (True, False, True)),
                                        ((3, 3, 3), (True, True, True))])
def test_lexicographic_ragged_boxes(orc, n, periodic):
    """The dense single kernel on boxes that are no multiple of its 64x4
    tile (partial tiles in x and y), with walls on a non-periodic axis."""
    _say(f"lex ragged {n} periodic={periodic}")
    rng = np.random.default_rng(sum(n))
    rho = 1 + 0.01 * rng.standard_normal((n[2], n[1], n[0]))
    u = 0.03 * rng.standard_normal((n[2], n[1], n[0], 3))
    faces = {}
    for a in range(3):
        if not periodic[a]:
            faces[2 * a] = (lbm.BC_BOUNCE_BACK, (0, 0, 0))
            faces[2 * a + 1] = (lbm.BC_MOVING_WALL, (0.05, 0.0, 0.0) if a != 0 else (0.0, 0.05, 0.0))
    ro, uo = oracle_run(orc, n, 40, rho, u, None, periodic, faces, 0.6)
    g, r, v, m0, m1 = gpu_run(n, 40, rho, u, None, periodic, faces, 0.6, kind=lbm.DENSE,
                              schedule=lbm.PLAIN_SINGLE_KERNEL)
    err = rel(v, uo)
    _say(f"  rel L2 u = {err:.3e}")
    assert err < 1e-5
    assert rel(r, ro) < 1e-6
    g.close()


def test_couette_one_voxel_wide_channel(orc):
    """1 x 16 x 1 periodic channel between a wall and a moving lid: the
    populations of the periodic axes stream onto themselves."""
    n, steps, uw = (1, 16, 1), 2000, 0.05
    faces = {lbm.YMIN: (lbm.BC_BOUNCE_BACK, (0, 0, 0)), lbm.YMAX: (lbm.BC_MOVING_WALL, (uw, 0.0, 0.0))}
    periodic = (True, False, True)
    rho = np.ones((1, 16, 1))
    u = np.zeros((1, 16, 1, 3))
    ro, uo = oracle_run(orc, n, steps, rho, u, None, periodic, faces, 1.0)
    g, r, v, m0, m1 = gpu_run(n, steps, rho, u, None, periodic, faces, 1.0, kind=lbm.DENSE,
                              schedule=lbm.PLAIN_SINGLE_KERNEL)
    err = rel(v, uo)
    lin = rel(v[:, 0], uw * (np.arange(16) + 0.5) / 16)
    _say(f"  rel L2 u vs oracle = {err:.3e}, vs linear profile = {lin:.3e}")
    assert err < 1e-5
    assert lin < 1e-4  # steady Couette flow is linear (halfway walls)
    assert abs(m1 - m0) / m0 < 1e-6
    g.close()


def test_single_block_grid(orc):
    """A 4^3 box: one block, every voxel on a wall, the lid on z+.  Dense
    (grouped, bitmask and lexicographic) and block-sparse (naive single
    kernel) arms agree bit for bit and with the oracle."""
    n, steps, tau = (4, 4, 4), 200, 0.55
    faces = {f: (lbm.BC_BOUNCE_BACK, (0, 0, 0)) for f in range(6)}
    faces[lbm.ZMAX] = (lbm.BC_MOVING_WALL, (0.1, 0.0, 0.0))
    periodic = (False,) * 3
    rho = np.ones((4, 4, 4))
    u = np.zeros((4, 4, 4, 3))
    ro, uo = oracle_run(orc, n, steps, rho, u, None, periodic, faces, tau)
    pops = []
    for kind, sch in ((lbm.DENSE, lbm.PLAIN_SINGLE_KERNEL), (lbm.DENSE, lbm.DISAGG),
                      (lbm.DENSE, lbm.DISAGG_BITMASK), (lbm.BLOCK_SPARSE, lbm.PLAIN_SINGLE_KERNEL),
                      (lbm.BLOCK_SPARSE, lbm.DISAGG)):
        fluid = np.ones((4, 4, 4), np.uint8) if kind == lbm.BLOCK_SPARSE else None
        g, r, v, m0, m1 = gpu_run(n, steps, rho, u, fluid, periodic, faces, tau, kind=kind, schedule=sch)
        err = rel(v, uo)
        _say(f"  kind={kind} schedule={sch}: rel L2 u = {err:.3e}, mass drift {abs(m1 - m0) / m0:.1e}")
        assert err < 1e-5
        assert abs(m1 - m0) / m0 < 1e-6
        if kind == lbm.DENSE and sch == lbm.DISAGG:
            _, gb, gm, gf, tot = g.index_map(lbm.MAP_GROUPS)
            assert (gb, gm, gf, tot) == (1, 0, 0, 1)
        pops.append(g.populations().cpu().numpy())
        g.close()
    for p in pops[1:]:
        assert np.array_equal(pops[0], p)


def test_isolated_fluid_voxels(orc):
    """Sparse grid whose fluid voxels have no fluid neighbour at all (one
    per active block, scattered) next to a few fluid clusters: every pull of
    an isolated voxel bounces back, so its density never changes."""
    n, steps = (16, 16, 16), 50
    rng = np.random.default_rng(3)
    fluid = np.zeros((16, 16, 16), np.uint8)
    iso = []
    for bz in range(4):
        for by in range(4):
            for bx in range(4):
                if (bx + by + bz) % 3 == 0 and not (bz == 2 and by == 0 and bx < 2):  # not in the cluster
                    z, y, x = bz * 4 + 1 + rng.integers(0, 2), by * 4 + 1 + rng.integers(0, 2), bx * 4 + 1 + rng.integers(0, 2)
                    fluid[z, y, x] = 1
                    iso.append((z, y, x))
    fluid[8:12, 0:4, 0:8] = 1  # a cluster (its own blocks)
    rho = 1 + 0.01 * rng.standard_normal((16, 16, 16))
    u = 0.03 * rng.standard_normal((16, 16, 16, 3))
    periodic = (True, True, True)
    ro, uo = oracle_run(orc, n, steps, rho, u, fluid, periodic, {}, 0.7)
    pops = []
    for sch in (lbm.PLAIN_SINGLE_KERNEL, lbm.DISAGG, lbm.DISAGG_BITMASK):
        g, r, v, m0, m1 = gpu_run(n, steps, rho, u, fluid, periodic, {}, 0.7, kind=lbm.BLOCK_SPARSE,
                                  schedule=sch)
        err = rel(v, uo)
        _say(f"  schedule={sch}: rel L2 u = {err:.3e}")
        assert err < 1e-5
        assert abs(m1 - m0) / m0 < 1e-6
        # isolated voxels keep their density (bounce-back and collision conserve it)
        fl_idx = np.flatnonzero(fluid.reshape(-1))
        pos = {int(k): i for i, k in enumerate(fl_idx)}
        for z, y, x in iso:
            k = pos[int(x + 16 * (y + 16 * z))]
            assert abs(r[k] - rho[z, y, x]) < 1e-5
        pops.append(g.populations().cpu().numpy())
        g.close()
    assert np.array_equal(pops[0], pops[1]) and np.array_equal(pops[0], pops[2])


@pytest.mark.parametrize("storage", [lbm.F32, lbm.F16_SHIFTED])
def test_check_reports_non_finite_populations(storage):
    """lbm_check passes on a healthy field and returns LBM_ERR_NUMERIC once
    one population is NaN (written through lbm_write_populations), and the
    NaN spreads through the steps without any kernel fault."""
    n = (16, 16, 16)
    g = lbm.Grid(*n, kind=lbm.DENSE, tau=0.6, storage=storage).bind()
    g.init_equilibrium(np.ones(16 ** 3), np.zeros((3, 16 ** 3)))
    g.step(5)
    g.check()
    f = g.populations()
    f[7, 1234] = float("nan")
    g.write_populations(f)
    with pytest.raises(lbm.LbmError) as e:
        g.check()
    assert e.value.status == -6
    g.step(3)
    with pytest.raises(lbm.LbmError):
        g.check()
    g.close()
