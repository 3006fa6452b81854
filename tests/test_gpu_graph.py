"""lbm_step inside a captured HIP graph (MI355X).

A step launches only kernels on the caller's stream (no allocation, no
memset, no host synchronization), so it can be captured: the graph holds
the launches of n steps with the buffer roles they had.  The roles cycle
(two buffers per dense or block-sparse level, three per multires level,
period at most 6 coarse steps), so a graph of a whole number of periods
replays as that many further steps.  Each replay is checked against a
second grid stepped eagerly, bit for bit, with the program's own eager work
and synchronization between replays.
"""
import sys

import numpy as np
import pytest

from paper_2503_07898_amd import cases, lbm, workloads

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


def _pops(g, levels):
    return [g.populations(level=l).cpu().numpy() for l in range(levels)]


def _replay_against_eager(make, levels, period, replays=4):
    ge, gg = make(), make()
    ge.step(period)  # eager warm-up on both (sizes the residency request outside the capture)
    gg.step(period)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gg.step(period)  # recorded, not run; the host roles come back to where they were
    torch.cuda.synchronize()
    for r in range(replays):
        graph.replay()
        ge.step(period)
        torch.cuda.synchronize()
        a, b = _pops(ge, levels), _pops(gg, levels)
        for l in range(levels):
            assert np.array_equal(a[l], b[l]), (r, l)
    ge.close()
    gg.close()


@pytest.mark.parametrize("storage", [lbm.F32, lbm.F16_SHIFTED])
def test_dense_cavity_graph_replays_bitwise(storage):
    _say(f"graph: cavity 48^3 storage={storage}")
    _replay_against_eager(lambda: cases.cavity(n=48, storage=storage), 1, 2)


def test_sparse_tunnel_graph_replays_bitwise():
    _say("graph: tunnel 64x32x32")

    def make():
        n = (64, 32, 32)
        fluid, _ = workloads.channel_packing(*n, seed=11, rmin=3.0, rmax=8.0, target_active=0.6)
        faces = {lbm.XMIN: (lbm.BC_REG_VELOCITY, (0.05, 0.0, 0.0)),
                 lbm.XMAX: (lbm.BC_REG_PRESSURE, (1.0, 0.0, 0.0))}
        for f in (lbm.YMIN, lbm.YMAX, lbm.ZMIN, lbm.ZMAX):
            faces[f] = (lbm.BC_BOUNCE_BACK, (0, 0, 0))
        g = lbm.Grid(*n, kind=lbm.BLOCK_SPARSE, fluid=fluid, periodic=(False,) * 3, faces=faces,
                     tau=0.6).bind()
        u = np.zeros((3, g.n))
        u[0] = 0.05
        g.init_equilibrium(np.ones(g.n), u)
        return g

    _replay_against_eager(make, 1, 2)


def test_multires_graph_replays_bitwise():
    _say("graph: multires cavity 64^3, 3 levels")
    _replay_against_eager(lambda: cases.multires_cavity(n=64), 3, 6)
