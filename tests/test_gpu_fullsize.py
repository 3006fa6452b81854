"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (MI355X).

Two kinds of check:
* whole-field runs: the dense cavity 256^3 and the block-sparse wind tunnel
  512x256x256 run 200 steps on the GPU and in the FP64 oracle (16 host
  threads, about a minute each) from the same initial state, and every fluid
  voxel's velocity is compared (1e-5 relative L2 for FP32 storage, 1e-2 for
  16-bit storage); the multires sphere runs whole coarse steps on both sides;
* one-step checks: the GPU runs some steps, its whole population field is
  read, the GPU advances one more step, and the oracle recomputes that step
  at sampled voxels (every corner, edge and face of the box, the inlet and
  outlet layers, voxels next to obstacles, random interior voxels), so each
  boundary rule is checked at full size against FP32 rounding of one step.
The wind tunnel also runs its full 1000 steps with both collision operators
and must stay finite with bounded mass.
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


def whole_field_oracle(orc, n, steps, fluid, faces, periodic, tau, u0):
    """FP64 oracle velocity in canonical order after `steps` steps from the
    equilibrium at rho = 1, u = u0 (fluid voxels)."""
    nx, ny, nz = n
    okind = {lbm.BC_BOUNCE_BACK: orc.BB, lbm.BC_MOVING_WALL: orc.MOVING,
             lbm.BC_REG_VELOCITY: orc.REG_VEL, lbm.BC_REG_PRESSURE: orc.REG_PRES}
    bc = [(orc.BB, (0, 0, 0))] * 6
    for f, (k, v) in faces.items():
        bc[f] = (okind[k], v)
    og = orc.Grid(nx, ny, nz, periodic=periodic, fluid=fluid, bc=bc, tau=tau)
    fl = np.ones((nz, ny, nx), bool) if fluid is None else np.asarray(fluid, bool)
    u = np.zeros((nz, ny, nx, 3))
    u[..., 0] = u0 * fl
    f = og.run(og.init_equilibrium(np.ones((nz, ny, nx)), u), steps)
    del u
    r, v = og.macroscopic(f)
    del f
    return r[fl], v[fl]


def whole_field_gpu(g, steps, u0):
    N = g.n
    u = np.zeros((3, N))
    u[0] = u0
    g.init_equilibrium(np.ones(N), u)
    g.step(steps)
    r, v = g.macroscopic()
    return r.cpu().numpy(), v.cpu().numpy().T


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def cavity_200(orc):
    _say("oracle: cavity 256^3, 200 steps")
    return whole_field_oracle(orc, (256, 256, 256), 200, None, cavity_faces(), (False,) * 3, 0.55, 0.0)


@pytest.mark.parametrize("storage,bar", [(lbm.F32, 1e-5), (lbm.F16_SHIFTED, 1e-2)])
def test_cavity_256_200_steps_whole_field(cavity_200, storage, bar):
    ro, uo = cavity_200
    _say(f"cavity 256^3, 200 steps, storage={storage}")
    g = lbm.Grid(256, 256, 256, kind=lbm.DENSE, periodic=(False,) * 3, faces=cavity_faces(), tau=0.55,
                 storage=storage).bind()
    r, v = whole_field_gpu(g, 200, 0.0)
    g.close()
    err = rel(v, uo)
    _say(f"  rel L2 u = {err:.3e}, rho - 1: {rel(r - 1, ro - 1):.3e}")
    assert err < bar


@pytest.fixture(scope="module")
def tunnel_200(orc):
    n, fluid, faces = tunnel_setup()
    _say("oracle: wind tunnel 512x256x256, 200 steps")
    return whole_field_oracle(orc, n, 200, fluid, faces, (False,) * 3, 0.6, 0.05)


@pytest.mark.parametrize("storage,schedule,bar", [
    (lbm.F32, lbm.DISAGG, 1e-5),
    (lbm.F32, lbm.DISAGG_BITMASK, 1e-5),
    (lbm.F16_SHIFTED, lbm.DISAGG, 1e-2),
    (lbm.BF16_SHIFTED, lbm.DISAGG, 1e-2),
])
def test_tunnel_200_steps_whole_field(tunnel_200, storage, schedule, bar):
    ro, uo = tunnel_200
    n, fluid, faces = tunnel_setup()
    _say(f"tunnel 512x256x256, 200 steps, storage={storage} schedule={schedule}")
    g = lbm.Grid(*n, kind=lbm.BLOCK_SPARSE, periodic=(False,) * 3, fluid=fluid, faces=faces, tau=0.6,
                 storage=storage, schedule=schedule).bind()
    r, v = whole_field_gpu(g, 200, 0.05)
    g.close()
    err = rel(v, uo)
    _say(f"  rel L2 u = {err:.3e}, rho - 1: {rel(r - 1, ro - 1):.3e}")
    assert err < bar


@pytest.mark.parametrize("collision", [lbm.BGK, lbm.REGULARIZED])
def test_tunnel_1000_steps_stays_finite(collision):
    """The wind tunnel's configured length: finite populations at every
    check, total mass within 5% of its initial value, speeds below 0.2."""
    n, fluid, faces = tunnel_setup()
    _say(f"tunnel 512x256x256, 1000 steps, collision={collision}")
    g = lbm.Grid(*n, kind=lbm.BLOCK_SPARSE, periodic=(False,) * 3, fluid=fluid, faces=faces, tau=0.6,
                 collision=collision).bind()
    N = g.n
    u = np.zeros((3, N))
    u[0] = 0.05
    g.init_equilibrium(np.ones(N), u)
    for k in range(10):
        g.step(100)
        g.check()  # raises on a NaN or infinite population
        m = g.reduce().cpu().numpy()
        _, v = g.macroscopic(f64=False)
        umax = float(v.norm(dim=0).max())
        _say(f"  step {100 * (k + 1)}: mass / N = {m[0] / N:.5f}, x-momentum / N = {m[1] / N:.5f}, "
             f"max |u| = {umax:.4f}")
        assert abs(m[0] / N - 1.0) < 0.05
        assert umax < 0.2
    g.close()


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
    fluid, _ = workloads.channel_packing(*n, seed=7898)
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


MR_STEPS = 10  # coarse steps (40 finest-level steps)


def multires_sphere_setup():
    n, levels = (512, 256, 256), 3
    lm, fluid = workloads.multires_sphere(*n, levels=levels)
    faces = {lbm.XMIN: (lbm.BC_REG_VELOCITY, (0.05, 0.0, 0.0)),
             lbm.XMAX: (lbm.BC_REG_PRESSURE, (1.0, 0.0, 0.0))}
    return n, levels, lm, fluid, faces


@pytest.fixture(scope="module")
def multires_sphere_ref(orc):
    n, levels, lm, fluid, _ = multires_sphere_setup()
    _say(f"oracle: multires sphere, {MR_STEPS} coarse steps")
    og = orc.MultiresGrid(*n, levels=levels, level_map=lm, fluid=fluid, periodic=(False, True, True),
                          bc=[(orc.REG_VEL, (0.05, 0, 0)), (orc.REG_PRES, (1.0, 0, 0))] + [(orc.BB, (0, 0, 0))] * 4,
                          tau_coarsest=0.52)
    rho = [np.ones(og.shape(l)) for l in range(levels)]
    u = []
    for l in range(levels):
        uu = np.zeros(og.shape(l) + (3,))
        uu[..., 0] = 0.05
        u.append(uu)
    f = og.run(og.init_equilibrium(rho, u), MR_STEPS)
    ref = og.macroscopic(f)
    del f
    return [ref[l][1][og.active(l)] for l in range(levels)]


@pytest.mark.parametrize("storage,bar", [(lbm.F32, 1e-5), (lbm.F16_SHIFTED, 1e-2)])
def test_multires_sphere_full_size_coarse_steps(multires_sphere_ref, storage, bar):
    """The 3-level sphere at its benchmark size (coarsest 128x64x64): whole
    coarse steps on GPU and oracle from the same state, all voxels."""
    n, levels, lm, fluid, faces = multires_sphere_setup()
    g = lbm.Grid(*n, kind=lbm.MULTIRES, levels=levels, level_map=lm, fluid=fluid, periodic=(False, True, True),
                 faces=faces, tau=0.52, storage=storage).bind()
    for l in range(levels):
        N = g.n_level(l)
        uu = np.zeros((3, N))
        uu[0] = 0.05
        g.init_equilibrium(np.ones(N), uu, level=l)
    g.step(MR_STEPS)
    for l in range(levels):
        _, v = g.macroscopic(level=l)
        v = v.cpu().numpy().T
        uref = multires_sphere_ref[l]
        du = v - uref
        # the deviation from the inflow state is the part the steps change
        dev = uref - np.array([0.05, 0, 0])
        err = np.linalg.norm(du) / max(np.linalg.norm(dev), 1e-30)
        err_u = np.linalg.norm(du) / np.linalg.norm(uref)
        _say(f"  storage {storage} level {l}: rel L2 u = {err_u:.2e}, of the change = {err:.2e}")
        assert err_u < bar
    g.close()
