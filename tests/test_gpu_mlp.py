"""GPU tests of the learned collision closure (MI355X).

* forward and gradients of the matrix-core network against the FP64 oracle
  evaluated on the same bf16-rounded weights and the same standardization
  (bar 1e-2: bf16 operands);
* training on the solver's own regularized populations lowers the loss;
* the closure in the solver conserves mass and stays within 1e-2 of the
  FP64 regularized operator on a Taylor-Green vortex, and a trained network
  does better than an untrained one (what the training gains).
"""
import math
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


@pytest.fixture(scope="module")
def mlpo(orc):
    from oracle import mlp
    return mlp


def populations(orc, n, seed, amp=0.03):
    rng = np.random.default_rng(seed)
    f = np.zeros((n, 19))
    for k in range(n):
        f[k] = orc.equilibrium(rng.uniform(0.97, 1.03), rng.uniform(-0.06, 0.06, 3))
        f[k] *= 1 + amp * rng.standard_normal(19)
    return f


def oracle_params(mlpo, W, stdz):
    s = np.asarray(stdz, np.float64)
    return mlpo.Params(*[np.asarray(w, np.float64) for w in W], in_mean=s[:19], in_std=1.0 / s[32:51],
                       out_std=s[64:83], out_mean=s[96:115]).bf16_rounded()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def test_forward_and_gradients_match_oracle(orc, mlpo):
    W = workloads.mlp_he_uniform(3)
    f = populations(orc, 1000, 1)
    m = lbm.Mlp()
    m.set_params(lbm.flatten_params(W))
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    m.fit_standardization(ft)
    stdz = m.standardization()
    # the oracle sees the same (float32) inputs, weights rounded to bf16
    p = oracle_params(mlpo, lbm.unflatten_params(m.params()), stdz)
    f32 = f.astype(np.float32).astype(np.float64)
    g = mlpo.closure_inputs(f32)
    y_ref = mlpo.forward(p, g)
    y = m.forward(ft).cpu().numpy()
    e = rel(y, y_ref)
    _say(f"  forward rel err {e:.2e}")
    assert e < 1e-2
    grads, loss = m.gradients(ft)
    t = mlpo.regularized_target(f32)
    ref = mlpo.backward(p, g, t)
    lr = mlpo.loss(p, g, t)
    _say(f"  loss gpu {loss.item():.6e} oracle {lr:.6e}")
    assert abs(loss.item() / lr - 1) < 1e-2
    gg = lbm.unflatten_params(grads.cpu().numpy())
    for name, a, b in zip(mlpo.Params.TRAINED, gg, ref):
        e = rel(a, b)
        _say(f"  grad {name} rel err {e:.2e}")
        assert e < 1e-2, name
    m.close()


@pytest.fixture(scope="module")
def closure_case():
    """A non-equilibrium state of a regularized Taylor-Green run (16^3) and a
    network standardized on samples of it."""
    n, tau = 16, 0.6
    rho, u = workloads.taylor_green_3d(n, 0.05)
    src = lbm.Grid(n, n, n, kind=lbm.DENSE, tau=tau, collision=lbm.REGULARIZED).bind()
    src.init_equilibrium(rho.reshape(-1), u.reshape(-1, 3).T.copy())
    src.step(5)
    f0 = src.populations().cpu().numpy()  # post-collision state [19][N]
    data = src.sample(1, 20_000)
    src.close()
    m = lbm.Mlp()
    m.set_params(lbm.flatten_params(workloads.mlp_he_uniform(9)))
    m.fit_standardization(data)
    yield n, tau, f0, m
    m.close()


def closure_step(orc, mlpo, closure_case, storage, judge):
    """One GPU step with the closure and the oracle's closure applied to the
    same stored (rounded) state: (gpu f*, oracle f*, oracle f^eq, fallbacks)."""
    n, tau, f0, m = closure_case
    m.set_judge(judge)
    g = lbm.Grid(n, n, n, kind=lbm.DENSE, tau=tau, storage=storage).bind()
    g.set_collision(lbm.MLP, m)
    g.write_populations(f0)
    start = g.populations().cpu().numpy()  # the stored (rounded) state
    m.fallbacks(reset=True)
    g.step(1)
    f1 = g.populations().cpu().numpy().T
    fb = m.fallbacks()
    g.close()
    c, _, _ = orc.lattice()
    pre = np.empty_like(start)
    for i in range(19):
        pre[i] = np.roll(start[i].reshape(n, n, n), shift=(c[i][2], c[i][1], c[i][0]),
                         axis=(0, 1, 2)).reshape(-1)
    p = oracle_params(mlpo, lbm.unflatten_params(m.params()), m.standardization())
    ref, fell = mlpo.collide(p, pre.T, tau, judge=judge)
    feq = np.array([orc.equilibrium(*orc.moments(ref[k])) for k in range(ref.shape[0])])
    return f1, ref, feq, fb, int(fell.sum()), fell.size


# bfloat16 storage rounds the stored h = f* - w to 8 significant bits; the
# compared part f* - f^eq is small next to h, so that rounding shows in it:
# 1.71e-2 measured against the 1e-2 bar (binary16: 4.0e-3), an expected
# failure.
@pytest.mark.parametrize("storage,judge", [
    (lbm.F32, 0.0), (lbm.F16_SHIFTED, 0.0),
    pytest.param(lbm.BF16_SHIFTED, 0.0, marks=pytest.mark.xfail(
        reason="bfloat16 storage: 1.71e-2 measured against the 1e-2 bar", strict=False)),
    (lbm.F32, 0.01),
])
def test_closure_step_matches_oracle(orc, mlpo, closure_case, storage, judge):
    """One solver step with the closure against the oracle's closure
    (stream, then collide with the same bf16-rounded weights), on a
    non-equilibrium state of a regularized Taylor-Green run."""
    f1, ref, feq, fb, fell, size = closure_step(orc, mlpo, closure_case, storage, judge)
    e = rel(f1 - feq, ref - feq)
    _say(f"  storage {storage} judge {judge}: rel L2 of f* - f^eq vs oracle closure {e:.2e}, "
         f"fallbacks gpu {fb} oracle {fell}")
    # decisions taken in different precisions may differ at the threshold
    assert abs(fb - fell) <= max(2, size // 200)
    assert e < 1e-2


@pytest.mark.parametrize("storage", [lbm.F32, lbm.F16_SHIFTED])
def test_closure_step_ragged_block_count(orc, mlpo, storage):
    """The closure on a 12^3 periodic box: 27 blocks, so the last workgroup
    of the kernel that takes two blocks per wave (16-bit storage) has waves
    with one block and waves with none.  One step against the oracle's
    closure, as above."""
    n, tau = 12, 0.6
    rho, u = workloads.taylor_green_3d(n, 0.05)
    src = lbm.Grid(n, n, n, kind=lbm.DENSE, tau=tau, collision=lbm.REGULARIZED).bind()
    src.init_equilibrium(rho.reshape(-1), u.reshape(-1, 3).T.copy())
    src.step(5)
    f0 = src.populations().cpu().numpy()
    data = src.sample(2, 20_000)
    src.close()
    m = lbm.Mlp()
    m.set_params(lbm.flatten_params(workloads.mlp_he_uniform(11)))
    m.fit_standardization(data)
    f1, ref, feq, fb, fell, size = closure_step(orc, mlpo, (n, tau, f0, m), storage, 0.0)
    m.close()
    e = rel(f1 - feq, ref - feq)
    _say(f"  12^3 storage {storage}: rel L2 of f* - f^eq vs oracle closure {e:.2e}, fallbacks gpu {fb} oracle {fell}")
    assert abs(fb - fell) <= max(2, size // 200)
    assert e < 1e-2


def _obstacle_box(n=24, r=5.0):
    """Periodic n^3 box with a solid sphere at the centre: full blocks away
    from it, bounce-masked blocks around it, no boundary group."""
    z, y, x = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")
    solid = (x - n / 2) ** 2 + (y - n / 2) ** 2 + (z - n / 2) ** 2 < r * r
    return (~solid).astype(np.uint8)


@pytest.mark.parametrize("storage", [lbm.F32, lbm.F16_SHIFTED])
def test_closure_masked_blocks_match_oracle(orc, mlpo, storage):
    """The closure on blocks next to an obstacle (the masked group, whose
    pulls bounce back where the source is solid): one step against the
    oracle's closure applied to the populations pulled with halfway
    bounce-back from the same stored state, and the 32-bit and 64-bit pull
    addressing bit for bit over four steps."""
    n, tau = 24, 0.6
    fluid = _obstacle_box(n)
    fb_mask = fluid.astype(bool)
    rho, u = workloads.taylor_green_3d(n, 0.05)
    u = u * fluid[..., None]
    geo = dict(kind=lbm.BLOCK_SPARSE, periodic=(True,) * 3, fluid=fluid, tau=tau)
    src = lbm.Grid(n, n, n, collision=lbm.REGULARIZED, **geo).bind()
    _, gb, gm, gf, _ = src.index_map(lbm.MAP_GROUPS)
    assert gb == 0 and gm > 0 and gf > 0
    src.init_equilibrium(rho[fb_mask], u[fb_mask].T.copy())
    src.step(5)
    f0 = src.populations().cpu().numpy()
    data = src.sample(3, 20_000)
    src.close()
    m = lbm.Mlp()
    m.set_params(lbm.flatten_params(workloads.mlp_he_uniform(13)))
    m.fit_standardization(data)
    m.set_judge(0.0)

    def run(wide, steps):
        g = lbm.Grid(n, n, n, storage=storage, **geo).bind()
        g.set_collision(lbm.MLP, m)
        g.set_wide_addressing(wide)
        g.write_populations(f0)
        start = g.populations().cpu().numpy()
        m.fallbacks(reset=True)
        g.step(steps)
        out = g.populations().cpu().numpy()
        fb = m.fallbacks()
        g.close()
        return start, out, fb

    _say(f"  masked closure: storage {storage}, {int(gm)} masked and {int(gf)} full blocks")
    start, f1, fb = run(False, 1)
    # pull with halfway bounce-back on the periodic box
    c, _, opp = orc.lattice()
    box = np.zeros((19, n, n, n))
    box[:, fb_mask] = start
    pre = np.empty_like(box)
    for i in range(19):
        sh = (c[i][2], c[i][1], c[i][0])
        src_fluid = np.roll(fb_mask, shift=sh, axis=(0, 1, 2))
        pre[i] = np.where(src_fluid, np.roll(box[i], shift=sh, axis=(0, 1, 2)), box[opp[i]])
    pre = pre[:, fb_mask].T
    p = oracle_params(mlpo, lbm.unflatten_params(m.params()), m.standardization())
    ref, fell = mlpo.collide(p, pre, tau, judge=0.0)
    feq = np.array([orc.equilibrium(*orc.moments(ref[k])) for k in range(ref.shape[0])])
    e = rel(f1.T - feq, ref - feq)
    _say(f"  masked closure: rel L2 of f* - f^eq vs oracle closure {e:.2e}, fallbacks gpu {fb} "
         f"oracle {int(fell.sum())}")
    assert abs(fb - int(fell.sum())) <= max(2, fell.size // 200)
    assert e < 1e-2
    a4, b4 = run(False, 4)[1], run(True, 4)[1]
    assert np.isfinite(a4).all()
    assert np.array_equal(a4.view(np.uint8), b4.view(np.uint8))
    m.close()


def regularized_tg_samples(n_samples, seed, n=32, steps=40):
    """Populations from a regularized-operator run of a 3D Taylor-Green vortex."""
    rho, u = workloads.taylor_green_3d(n, 0.05)
    tau = workloads.tau_for_reynolds(200.0, 0.05, 2 * math.pi / n)
    g = lbm.Grid(n, n, n, kind=lbm.DENSE, tau=tau, collision=lbm.REGULARIZED).bind()
    g.init_equilibrium(rho.reshape(-1), u.reshape(-1, 3).T.copy())
    out = []
    per = n_samples // 4
    for k in range(4):
        g.step(steps // 4)
        out.append(g.sample(seed + k, per))
    g.close()
    return torch.cat(out)


def train(m, data, iters, batch=4096, lr=1e-3, seed=0):
    rng = np.random.default_rng(seed)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    hist = []
    for t in range(1, iters + 1):
        idx = torch.as_tensor(rng.integers(0, data.shape[0], batch), device="cuda")
        lr_t = 1e-5 + 0.5 * (lr - 1e-5) * (1 + math.cos(math.pi * (t - 1) / iters))
        m.train_step(data, lr_t, t, loss, idx=idx)
        if t % max(1, iters // 10) == 0 or t == 1:
            hist.append(loss.item())
    return hist


def test_training_lowers_loss():
    data = regularized_tg_samples(200_000, 7)
    m = lbm.Mlp()
    m.set_params(lbm.flatten_params(workloads.mlp_he_uniform(11)))
    m.fit_standardization(data)
    hist = train(m, data, 400)
    _say(f"  loss history {['%.3e' % h for h in hist]}")
    assert hist[-1] < 0.1 * hist[0]
    m.close()


def test_adam_on_caller_gradients_equals_train_step():
    """lbm_mlp_gradients + lbm_mlp_adam(grads) gives the same weights, bit
    for bit, as lbm_mlp_train_step on the same batches."""
    data = regularized_tg_samples(20_000, 3)
    nets = []
    for _ in range(2):
        m = lbm.Mlp()
        m.set_params(lbm.flatten_params(workloads.mlp_he_uniform(5)))
        m.fit_standardization(data)
        nets.append(m)
    for t in range(1, 6):
        batch = data[(t - 1) * 4096:t * 4096]
        nets[0].train_step(batch, 1e-3, t)
        g, _ = nets[1].gradients(batch)
        nets[1].adam(g, 1e-3, t)
    a, b = nets[0].params(), nets[1].params()
    assert np.array_equal(a, b)
    assert not np.array_equal(a, lbm.flatten_params(workloads.mlp_he_uniform(5)))
    for m in nets:
        m.close()


def splitmix64(x):
    """splitmix64 (Steele, Lea and Flood 2014) on Python integers."""
    mask = (1 << 64) - 1
    x = (x + 0x9E3779B97F4A7C15) & mask
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & mask
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & mask
    return x ^ (x >> 31)


def test_seeded_init_on_device():
    """lbm_mlp_init_params(seed): He-uniform weights per layer from the
    counter-based generator, zero biases; the same seed gives the same
    network, another seed another one."""
    m = lbm.Mlp()
    seed = 7898
    m.init_params(seed)
    p = m.params()
    l19, l64 = 0.5619514869490163, 0.30618621784789724  # sqrt(6/19), sqrt(6/64) in double
    lim = [l19] * (19 * 64) + [0.0] * 64 + [l64] * (64 * 64) + [0.0] * 64 + [l64] * (64 * 19) + [0.0] * 19
    want = np.empty(lbm.MLP_PARAMS, np.float32)
    for k in range(lbm.MLP_PARAMS):
        r = splitmix64(seed ^ splitmix64(k))
        u = (r >> 11) * (1.0 / 9007199254740992.0)
        want[k] = np.float32((2.0 * u - 1.0) * lim[k])
    assert np.array_equal(p, want)
    W = lbm.unflatten_params(p)
    for w, fan_in in ((W[0], 19), (W[2], 64), (W[4], 64)):
        assert np.abs(w).max() <= math.sqrt(6 / fan_in) and w.std() > 0.5 * math.sqrt(2 / fan_in)
    m.init_params(seed)
    assert np.array_equal(m.params(), p)
    m.init_params(seed + 1)
    assert not np.array_equal(m.params(), p)
    m.close()


def test_closure_in_solver(orc):
    """Taylor-Green at tau 0.5038 (Re 200 on 32^3), closure trained briefly on
    the solver's own regularized populations, run-time judge at its default
    (1%): within 1e-2 of the FP64 regularized operator, mass conserved, and
    the trained network keeps more of its own updates than the untrained one.
    Without the judge the errors are reported (near tau = 1/2 an overshoot of
    the regularized stress above 1.5% is unstable)."""
    n = 32
    data = regularized_tg_samples(200_000, 3)
    m = lbm.Mlp()
    m.set_params(lbm.flatten_params(workloads.mlp_he_uniform(5)))
    m.fit_standardization(data)
    untrained = lbm.Mlp()
    untrained.set_params(m.params())
    untrained.set_standardization(m.standardization())
    train(m, data, 600)
    rho, u = workloads.taylor_green_3d(n, 0.05)
    tau = workloads.tau_for_reynolds(200.0, 0.05, 2 * math.pi / n)
    steps = 60
    og = orc.Grid(n, n, n, tau=tau, collision=orc.REGULARIZED)
    fo = og.run(og.init_equilibrium(rho, u), steps)
    _, uo = og.macroscopic(fo)
    uo = uo.reshape(-1, 3)
    errs, fbs = {}, {}
    for name, net, coll, judge in (("mlp", m, lbm.MLP, 0.01), ("untrained", untrained, lbm.MLP, 0.01),
                                   ("mlp_nojudge", m, lbm.MLP, 0.0), ("bgk", None, lbm.BGK, 0.0)):
        if net is not None:
            net.set_judge(judge)
        g = lbm.Grid(n, n, n, kind=lbm.DENSE, tau=tau).bind()
        g.set_collision(coll, net)
        g.init_equilibrium(rho.reshape(-1), u.reshape(-1, 3).T.copy())
        m0 = g.reduce().cpu().numpy()[0]
        if net is not None:
            net.fallbacks(reset=True)
        g.step(steps)
        m1 = g.reduce().cpu().numpy()[0]
        _, v = g.macroscopic()
        v = v.cpu().numpy().T
        errs[name] = rel(v, uo) if np.all(np.isfinite(v)) else float("inf")
        fb = net.fallbacks() if net is not None else 0
        fbs[name] = fb / (n ** 3 * steps)
        _say(f"  {name}: rel L2 u vs FP64 regularized = {errs[name]:.3e}, mass drift "
             f"{abs(m1 - m0) / m0:.1e}, fallback fraction {fbs[name]:.3f}")
        if name == "mlp":
            assert abs(m1 - m0) / m0 < 1e-6
        g.close()
    assert errs["mlp"] < 1e-2
    assert fbs["mlp"] <= fbs["untrained"]
    m.close()
    untrained.close()


@pytest.mark.parametrize("case", ["taylor_green", "cavity"])
@pytest.mark.parametrize("storage", [lbm.F32, lbm.F16_SHIFTED, lbm.BF16_SHIFTED])
def test_closure_addressing_forms_bitwise(case, storage):
    """The closure kernel's 32-bit pull offsets (buffers up to 4 GiB) and its
    64-bit slot arithmetic (larger buffers, forced here) give the same
    populations bit for bit and the same fallback count: periodic
    Taylor-Green 32^3 (full blocks only) and a lid-driven cavity 32^3 (full
    blocks inside a boundary shell that runs the regularized operator),
    trained weights, judge on, 4 steps.  The masked blocks' form is held the
    same way in test_closure_masked_blocks_match_oracle."""
    from paper_2503_07898_amd import cases, train_closure
    w = train_closure.load()
    if w is None:
        pytest.skip("no trained closure weights in the package")
    net = lbm.Mlp()
    net.set_params(w[0])
    net.set_standardization(w[1])
    net.set_judge(0.01)
    out = {}
    for wide in (False, True):
        _say(f"  closure addressing: {case} storage={storage} wide={wide}")
        if case == "cavity":
            g = cases.cavity(n=32, storage=storage, tau=0.52)
        else:
            g = cases.taylor_green(n=32, re=400.0, storage=storage)
        g.set_collision(lbm.MLP, net)
        g.set_wide_addressing(wide)
        net.fallbacks(reset=True)
        g.step(4)
        torch.cuda.synchronize()
        out[wide] = (g.populations().cpu().numpy(), net.fallbacks())
        g.close()
    net.close()
    a, b = out[False], out[True]
    assert np.isfinite(a[0]).all()
    assert np.array_equal(a[0].view(np.uint8), b[0].view(np.uint8))
    assert a[1] == b[1]
