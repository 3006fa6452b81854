"""GPU parity of the D3Q27 path against the D3Q27 build of the FP64 oracle
(MI355X): dense Taylor-Green (FP32 1e-5, FP16 1e-2, BGK and regularized),
the lid-driven cavity and the block-sparse wind tunnel with regularized
inlet/outlet; the naive single kernel, the memory-grouped kernels and the
bitmask-grouped kernels must agree bit for bit."""
import sys

import numpy as np
import pytest

from paper_2503_07898_amd import lbm, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
Q27 = 27


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


def run_gpu(n, steps, rho, u, fluid=None, **kw):
    g = lbm.Grid(*n, fluid=fluid, q=Q27, **kw).bind()
    g.init_equilibrium(canon(rho, fluid), canon(u, fluid).T.copy())
    g.step(steps)
    r, v = g.macroscopic()
    return g, r.cpu().numpy(), v.cpu().numpy().T


def run_oracle(orc, n, steps, rho, u, fluid=None, periodic=(True,) * 3, faces=None, tau=0.6, collision=0):
    bc = [(orc.BB, (0, 0, 0))] * 6
    kind = {lbm.BC_BOUNCE_BACK: orc.BB, lbm.BC_MOVING_WALL: orc.MOVING,
            lbm.BC_REG_VELOCITY: orc.REG_VEL, lbm.BC_REG_PRESSURE: orc.REG_PRES}
    for f, (k, v) in (faces or {}).items():
        bc[f] = (kind[k], v)
    g = orc.Grid(*n, periodic=periodic, fluid=fluid, bc=bc, tau=tau, collision=collision, q=Q27)
    f = g.run(g.init_equilibrium(rho, u), steps)
    r, v = g.macroscopic(f)
    return canon(r, fluid), canon(v, fluid)


@pytest.mark.parametrize("collision", [lbm.BGK, lbm.REGULARIZED])
@pytest.mark.parametrize("storage,bar", [(lbm.F32, 1e-5), (lbm.F16_SHIFTED, 1e-2)])
def test_taylor_green_d3q27(orc, storage, bar, collision):
    n = 32
    rho, u = workloads.taylor_green_3d(n, 0.05)
    ro, uo = run_oracle(orc, (n,) * 3, 60, rho, u, tau=0.56, collision=collision)
    pops = []
    for sch in (lbm.PLAIN_SINGLE_KERNEL, lbm.DISAGG):
        g, r, v = run_gpu((n,) * 3, 60, rho, u, kind=lbm.DENSE, tau=0.56, storage=storage,
                          collision=collision, schedule=sch)
        err = rel(v, uo)
        _say(f"  TG D3Q27 storage={storage} coll={collision} schedule={sch}: rel L2 u = {err:.3e}")
        assert err < bar
        pops.append(g.populations().cpu().numpy())
        g.close()
    assert np.array_equal(pops[0], pops[1])


def test_cavity_d3q27(orc):
    n, steps, tau = (24, 24, 24), 200, 0.55
    rho = np.ones((n[2], n[1], n[0]))
    u = np.zeros(rho.shape + (3,))
    faces = {f: (lbm.BC_BOUNCE_BACK, (0, 0, 0)) for f in range(6)}
    faces[lbm.ZMAX] = (lbm.BC_MOVING_WALL, (0.1, 0.0, 0.0))
    ro, uo = run_oracle(orc, n, steps, rho, u, periodic=(False,) * 3, faces=faces, tau=tau)
    pops = []
    for sch in (lbm.PLAIN_SINGLE_KERNEL, lbm.DISAGG, lbm.DISAGG_BITMASK):
        g, r, v = run_gpu(n, steps, rho, u, kind=lbm.DENSE, periodic=(False,) * 3, faces=faces, tau=tau,
                          schedule=sch)
        err = rel(v, uo)
        _say(f"  cavity D3Q27 schedule={sch}: rel L2 u = {err:.3e}")
        assert err < 1e-5
        m = g.reduce().cpu().numpy()[0]
        assert abs(m - rho.sum()) / rho.sum() < 1e-6
        pops.append(g.populations().cpu().numpy())
        g.close()
    assert np.array_equal(pops[0], pops[1]) and np.array_equal(pops[0], pops[2])


@pytest.mark.parametrize("storage,bar", [(lbm.F32, 1e-5), (lbm.F16_SHIFTED, 1e-2), (lbm.BF16_SHIFTED, 1e-2)])
def test_sparse_tunnel_d3q27(orc, storage, bar):
    n, steps, tau = (64, 32, 32), 120, 0.6
    fluid, _ = workloads.sphere_packing(*n, seed=7, rmin=3.0, rmax=8.0, target_active=0.6)
    faces = {lbm.XMIN: (lbm.BC_REG_VELOCITY, (0.05, 0.0, 0.0)),
             lbm.XMAX: (lbm.BC_REG_PRESSURE, (1.0, 0.0, 0.0))}
    for f in (lbm.YMIN, lbm.YMAX, lbm.ZMIN, lbm.ZMAX):
        faces[f] = (lbm.BC_BOUNCE_BACK, (0, 0, 0))
    rho = np.ones((n[2], n[1], n[0]))
    u = np.zeros(rho.shape + (3,))
    u[..., 0] = 0.05 * fluid
    ro, uo = run_oracle(orc, n, steps, rho, u, fluid=fluid, periodic=(False,) * 3, faces=faces, tau=tau)
    pops = []
    for sch in (lbm.PLAIN_SINGLE_KERNEL, lbm.DISAGG, lbm.DISAGG_BITMASK):
        g, r, v = run_gpu(n, steps, rho, u, fluid=fluid, kind=lbm.BLOCK_SPARSE, periodic=(False,) * 3,
                          faces=faces, tau=tau, storage=storage, schedule=sch)
        err = rel(v, uo)
        _say(f"  tunnel D3Q27 storage={storage} schedule={sch}: rel L2 u = {err:.3e}")
        assert err < bar
        pops.append(g.populations().cpu().numpy())
        g.close()
    assert np.array_equal(pops[0], pops[1]) and np.array_equal(pops[0], pops[2])
