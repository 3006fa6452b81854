"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (MI355X).

The FP64 oracle cannot run these grids for many steps, so each test runs the
GPU for some steps, reads the whole population field, advances the GPU one
more step, and has the oracle recompute that step at sampled voxels (every
corner, edge and face of the box, the inlet/outlet layers, voxels next to
obstacles, and random interior voxels).  FP32 storage must agree to FP32
rounding of one step; 16-bit storage to its own rounding.  The multires
sphere runs whole coarse steps on both sides at full size.
"""
import sys

import numpy as np
import pytest

from paper_2503_07898_amd import lbm, workloads

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


def sample_voxels(n, fluid, rng, n_random=20000):
    nx, ny, nz = n
    fl = np.ones((nz, ny, nx), bool) if fluid is None else np.asarray(fluid, bool)
    pick = np.zeros((nz, ny, nx), bool)
    # faces, edges and corners of the box
    pick[[0, -1], :, :] |= rng.random((2, ny, nx)) < 0.05
    pick[:, [0, -1], :] |= rng.random((nz, 2, nx)) < 0.05
    pick[:, :, [0, -1]] |= rng.random((nz, ny, 2)) < 0.05
    for z in (0, nz - 1):
        for y in (0, ny - 1):
            pick[z, y, :] = True
        for x in (0, nx - 1):
            pick[z, :, x] = True
    for y in (0, ny - 1):
        for x in (0, nx - 1):
            pick[:, y, x] = True
    # fluid voxels touching a solid voxel
    if fluid is not None:
        near = np.zeros_like(fl)
        for ax in range(3):
            for sh in (-1, 1):
                near |= ~np.roll(fl, sh, axis=ax)
        cand = np.flatnonzero(near & fl)
        pick.reshape(-1)[rng.choice(cand, min(len(cand), n_random), replace=False)] = True
    cand = np.flatnonzero(fl)
    pick.reshape(-1)[rng.choice(cand, min(len(cand), n_random), replace=False)] = True
    return np.flatnonzero(pick & fl)


def one_step_check(orc, g, n, fluid, faces, periodic, tau, collision, storage, warm, seed):
    nx, ny, nz = n
    g.step(warm)
    f0 = g.populations().cpu().numpy()  # [19][N] FP64 images of the stored values
    g.step(1)
    f1 = g.populations().cpu().numpy()
    torch.cuda.synchronize()
    fl = np.ones((nz, ny, nx), bool) if fluid is None else np.asarray(fluid, bool)
    lin = np.flatnonzero(fl)
    box = np.zeros((nz * ny * nx, 19))
    box[lin] = f0.T
    del f0
    box = box.reshape(nz, ny, nx, 19)
    okind = {lbm.BC_BOUNCE_BACK: orc.BB, lbm.BC_MOVING_WALL: orc.MOVING,
             lbm.BC_REG_VELOCITY: orc.REG_VEL, lbm.BC_REG_PRESSURE: orc.REG_PRES}
    bc = [(orc.BB, (0, 0, 0))] * 6
    for f, (k, v) in faces.items():
        bc[f] = (okind[k], v)
    og = orc.Grid(nx, ny, nz, periodic=periodic, fluid=None if fluid is None else fluid, bc=bc, tau=tau,
                  collision=collision)
    rng = np.random.default_rng(seed)
    vox = sample_voxels(n, fluid, rng)
    ref = og.step_voxels(box, vox)
    canon = np.searchsorted(lin, vox)
    got = f1[:, canon].T
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    # compare the shifted populations f - w, the quantity the storage keeps
    err = np.abs(got - ref)
    scale = np.abs(ref - w).max()
    rel_max = err.max() / scale
    rel_l2 = np.linalg.norm(got - ref) / np.linalg.norm(ref - w)
    _say(f"  {len(vox)} sampled voxels: max |diff| / max |f - w| = {rel_max:.2e}, rel L2 = {rel_l2:.2e}")
    return rel_max, rel_l2


def cavity_faces():
    faces = {f: (lbm.BC_BOUNCE_BACK, (0, 0, 0)) for f in range(6)}
    faces[lbm.ZMAX] = (lbm.BC_MOVING_WALL, (0.1, 0.0, 0.0))
    return faces


@pytest.mark.parametrize("schedule", [lbm.DISAGG, lbm.PLAIN_SINGLE_KERNEL])
def test_cavity_256_one_step_sampled(orc, schedule):
    n = (256, 256, 256)
    _say(f"cavity 256^3 schedule={schedule}")
    faces = cavity_faces()
    g = lbm.Grid(*n, kind=lbm.DENSE, periodic=(False,) * 3, faces=faces, tau=0.55, schedule=schedule).bind()
    N = g.n
    g.init_equilibrium(np.ones(N), np.zeros((3, N)))
    rel_max, rel_l2 = one_step_check(orc, g, n, None, faces, (False,) * 3, 0.55, 0, lbm.F32, 30, 1)
    assert rel_max < 1e-5 and rel_l2 < 1e-6
    g.close()


def tunnel_setup():
    n = (512, 256, 256)
    fluid, _ = workloads.sphere_packing(*n, seed=7898)
    faces = {lbm.XMIN: (lbm.BC_REG_VELOCITY, (0.05, 0.0, 0.0)),
             lbm.XMAX: (lbm.BC_REG_PRESSURE, (1.0, 0.0, 0.0))}
    for f in (lbm.YMIN, lbm.YMAX, lbm.ZMIN, lbm.ZMAX):
        faces[f] = (lbm.BC_BOUNCE_BACK, (0, 0, 0))
    return n, fluid, faces


@pytest.mark.parametrize("storage,schedule,bars", [
    (lbm.F32, lbm.DISAGG, (1e-5, 1e-6)),
    (lbm.F32, lbm.PLAIN_SINGLE_KERNEL, (1e-5, 1e-6)),
    (lbm.F16_SHIFTED, lbm.DISAGG, (2e-3, 5e-4)),  # one binary16 rounding of f - w
])
def test_tunnel_512x256x256_one_step_sampled(orc, storage, schedule, bars):
    n, fluid, faces = tunnel_setup()
    _say(f"tunnel 512x256x256 storage={storage} schedule={schedule}")
    g = lbm.Grid(*n, kind=lbm.BLOCK_SPARSE, periodic=(False,) * 3, fluid=fluid, faces=faces, tau=0.6,
                 storage=storage, schedule=schedule).bind()
    N = g.n
    u = np.zeros((3, N))
    u[0] = 0.05
    g.init_equilibrium(np.ones(N), u)
    rel_max, rel_l2 = one_step_check(orc, g, n, fluid, faces, (False,) * 3, 0.6, 0, storage, 20, 2)
    assert rel_max < bars[0] and rel_l2 < bars[1]
    g.close()


def test_multires_sphere_full_size_coarse_steps(orc):
    """The 3-level sphere at its benchmark size (coarsest 128x64x64): a few
    whole coarse steps on GPU and oracle from the same state, all voxels."""
    n, levels = (512, 256, 256), 3
    lm, fluid = workloads.multires_sphere(*n, levels=levels)
    faces = {lbm.XMIN: (lbm.BC_REG_VELOCITY, (0.05, 0.0, 0.0)),
             lbm.XMAX: (lbm.BC_REG_PRESSURE, (1.0, 0.0, 0.0))}
    og = orc.MultiresGrid(*n, levels=levels, level_map=lm, fluid=fluid, periodic=(False, True, True),
                          bc=[(orc.REG_VEL, (0.05, 0, 0)), (orc.REG_PRES, (1.0, 0, 0))] + [(orc.BB, (0, 0, 0))] * 4,
                          tau_coarsest=0.52)
    rho = [np.ones(og.shape(l)) for l in range(levels)]
    u = []
    for l in range(levels):
        uu = np.zeros(og.shape(l) + (3,))
        uu[..., 0] = 0.05
        u.append(uu)
    steps = 3
    f = og.run(og.init_equilibrium(rho, u), steps)
    ref = og.macroscopic(f)
    del f
    g = lbm.Grid(*n, kind=lbm.MULTIRES, levels=levels, level_map=lm, fluid=fluid, periodic=(False, True, True),
                 faces=faces, tau=0.52).bind()
    for l in range(levels):
        N = g.n_level(l)
        uu = np.zeros((3, N))
        uu[0] = 0.05
        g.init_equilibrium(np.ones(N), uu, level=l)
    g.step(steps)
    for l in range(levels):
        a = og.active(l)
        _, v = g.macroscopic(level=l)
        v = v.cpu().numpy().T
        uref = ref[l][1][a]
        du = v - uref
        # compare the deviation from the inflow state, the part the steps change
        dev = uref - np.array([0.05, 0, 0])
        err = np.linalg.norm(du) / max(np.linalg.norm(dev), 1e-30)
        err_u = np.linalg.norm(du) / np.linalg.norm(uref)
        _say(f"  level {l}: rel L2 u = {err_u:.2e}, of the change = {err:.2e}")
        assert err_u < 1e-5
    g.close()
