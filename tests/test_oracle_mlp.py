"""Pins of the FP64 closure oracle (CPU): gradients against central finite
differences, the projection's exact moments, GELU against its derivative and
the erf form it approximates, the closure assembly against the regularized
operator, and Adam's closed-form first step."""
import math

import numpy as np
import pytest

from paper_2503_07898_amd import workloads


@pytest.fixture(scope="module")
def mlp(orc):
    from oracle import mlp
    return mlp


def make_params(mlp, seed=0):
    W = workloads.mlp_he_uniform(seed)
    rng = np.random.default_rng(seed + 1)
    for k in (1, 3, 5):
        W[k] = 0.1 * rng.standard_normal(W[k].shape)
    return mlp.Params(*W, in_mean=0.01 * rng.standard_normal(19), in_std=0.5 + rng.random(19),
                      out_mean=1e-3 * rng.standard_normal(19), out_std=0.01 + 0.02 * rng.random(19))


def sample_populations(orc, n, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    f = np.zeros((n, 19))
    for k in range(n):
        f[k] = orc.equilibrium(rng.uniform(0.95, 1.05), rng.uniform(-0.08, 0.08, 3))
        f[k] *= 1 + amp * rng.standard_normal(19)
    return f


def test_gradients_match_central_differences(orc, mlp):
    p = make_params(mlp)
    f = sample_populations(orc, 6, 1)
    g = mlp.closure_inputs(f)
    t = mlp.regularized_target(f)
    grads = mlp.backward(p, g, t)
    h = 1e-6
    for name, gr in zip(mlp.Params.TRAINED, grads):
        w = getattr(p, name)
        num = np.zeros_like(w)
        flat = w.reshape(-1)
        nf = num.reshape(-1)
        for k in range(flat.size):
            old = flat[k]
            flat[k] = old + h
            lp = mlp.loss(p, g, t)
            flat[k] = old - h
            lm = mlp.loss(p, g, t)
            flat[k] = old
            nf[k] = (lp - lm) / (2 * h)
        err = np.linalg.norm(num - gr) / max(np.linalg.norm(gr), 1e-30)
        assert err < 1e-6, (name, err)


def test_projection_moments_and_idempotence(orc, mlp):
    c, w = mlp.lattice()
    rng = np.random.default_rng(2)
    y = rng.standard_normal((50, 19))
    py = mlp.project(y)
    assert np.max(np.abs(py.sum(-1))) < 1e-14
    assert np.max(np.abs(py @ c)) < 1e-14
    assert np.allclose(mlp.project(py), py, atol=1e-14, rtol=0)
    # the regularized target already carries no mass or momentum
    f = sample_populations(orc, 20, 3)
    t = mlp.regularized_target(f)
    assert np.allclose(mlp.project(t), t, atol=1e-16, rtol=0)
    # P as a matrix equals P as a function
    assert np.allclose(y @ mlp.projection_matrix().T, py, atol=1e-14, rtol=0)
    # P keeps exactly the 6-dimensional second-order Hermite space: projecting
    # a non-equilibrium part gives the regularized operator's f1 (the C
    # oracle's own projection), and the 13 other w-orthogonal modes vanish
    assert np.linalg.matrix_rank(mlp.projection_matrix(), tol=1e-12) == 6
    g = mlp.closure_inputs(f)
    assert np.allclose(mlp.project(g), t, atol=1e-15, rtol=0)
    cubic = w * (c[:, 0] * c[:, 1] ** 2)  # a third-order (ghost) moment direction
    assert np.max(np.abs(mlp.project(cubic))) < 1e-16


def test_gelu(mlp):
    x = np.linspace(-6, 6, 241)
    h = 1e-6
    num = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(num - mlp.gelu_grad(x))) < 1e-8
    exact = np.array([0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in x])
    assert np.max(np.abs(mlp.gelu(x) - exact)) < 1e-3  # the tanh form's known accuracy


def test_closure_assembly_equals_regularized_with_exact_output(orc, mlp):
    p = make_params(mlp)
    p.in_std[:] = 1e3  # keep inputs far inside the fallback limit
    f = sample_populations(orc, 12, 4)
    t = mlp.regularized_target(f)
    for tau in (0.51, 0.6, 0.9):
        out, fell = mlp.collide(p, f, tau, y_override=t)
        assert not fell.any()
        ref = np.array([orc.collide_regularized(fk, tau) for fk in f])
        assert np.max(np.abs(out - ref)) < 1e-15


def test_closure_fallback_and_conservation(orc, mlp):
    p = make_params(mlp)
    f = sample_populations(orc, 30, 5, amp=0.1)
    out, fell = mlp.collide(p, f, 0.6)
    c, _ = mlp.lattice()
    assert np.allclose(out.sum(-1), f.sum(-1), atol=1e-14, rtol=0)
    assert np.allclose(out @ c, f @ c, atol=1e-14, rtol=0)
    p.in_std[:] = 1e-4  # every standardized input is huge -> every voxel falls back
    out2, fell2 = mlp.collide(p, f, 0.6)
    assert fell2.all()
    ref = np.array([orc.collide_regularized(fk, 0.6) for fk in f])
    assert np.max(np.abs(out2 - ref)) < 1e-16


def test_adam_first_step_closed_form(mlp):
    rng = np.random.default_rng(6)
    w = [rng.standard_normal((5, 4))]
    g = [rng.standard_normal((5, 4))]
    w0 = w[0].copy()
    opt = mlp.Adam(lr=1e-3)
    m, v = [np.zeros_like(w[0])], [np.zeros_like(w[0])]
    opt.step(w, g, m, v, 1)
    assert np.allclose(w[0], w0 - 1e-3 * g[0] / (np.abs(g[0]) + 1e-8), atol=1e-15, rtol=0)


def test_bf16_rounding_reference(mlp):
    # nearest-even at the 8th significant bit, checked on hand-picked values
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.14159265])
    out = mlp.bf16_round(vals)
    assert out[0] == 1.0
    assert out[1] == 1.0                    # tie -> even mantissa
    assert out[2] == 1.0 + 2 ** -6          # tie -> even (up)
    assert out[3] == -2.5
    assert out[4] == 3.140625


def test_closure_judge_threshold(orc, mlp):
    """The regularized operator judges the closure: an output within 1% (L2)
    of its non-equilibrium part is accepted, one 2% off falls back, and
    judge = 0 accepts both."""
    p = make_params(mlp)
    p.in_std[:] = 1e3  # inputs far inside the range limit
    p.out_std[:] = 1e-12  # a negligible absolute floor
    f = sample_populations(orc, 10, 6)
    t = mlp.regularized_target(f)
    for scale, judge, expect_fall in ((1.005, 0.01, False), (1.02, 0.01, True), (1.02, 0.0, False)):
        out, fell = mlp.collide(p, f, 0.51, y_override=t * scale, judge=judge)
        assert (fell == expect_fall).all(), (scale, judge)
        if not expect_fall:
            rho = f.sum(-1)
            feq = np.array([orc.equilibrium(*orc.moments(fk)) for fk in f])
            assert np.allclose(out, feq + (1 - 1 / 0.51) * rho[:, None] * t * scale, atol=1e-15, rtol=0)


def test_closure_judge_floor_near_equilibrium(orc, mlp):
    """At equilibrium f1 = 0: an output deviating by less than judge x floor
    (floor = |out_std|, the typical target size) is kept, a larger one falls
    back."""
    p = make_params(mlp)
    p.in_std[:] = 1e3
    p.out_std[:] = 1e-3
    f = np.array([orc.equilibrium(1.0 + 0.01 * k, [0.02, -0.01, 0.005 * k]) for k in range(5)])
    c, w = mlp.lattice()
    Qt = mlp.hermite_tensors()
    y = 4.5 * w * np.einsum("iab,ab->i", Qt, np.diag([1.0, -1.0, 0.0]))  # a pure stress direction
    lim = 0.01 * np.sqrt(np.sum(p.out_std ** 2))
    for size, expect_fall in ((0.5 * lim, False), (2.0 * lim, True)):
        yo = np.tile(y / np.linalg.norm(y) * size, (len(f), 1))
        _, fell = mlp.collide(p, f, 0.6, y_override=yo)
        assert (fell == expect_fall).all(), size


def test_forward_hand_computed_saturated_network(mlp):
    """forward() on a network built so that every pre-activation is 0 or
    +-15 / +-30: there the tanh-form GELU is exactly ReLU in FP64 (tanh
    saturates to +-1 beyond |t| ~ 19), so the output follows from the
    wiring alone.  The wiring uses shifts of the unit index (non-symmetric
    weight matrices), a bias unit and non-trivial standardization, so a
    transposed weight matrix, a misplaced bias or a standardization applied
    the wrong way round changes the result.

    Wiring (x = standardized input, entries in {-1, 0, 1}):
      layer 1: unit j < 19 sees 30 x_j; unit 63 is a bias unit (b1 = 30);
               unit 51 sees 30 x_1 - 15 (x_1 = -1: silent);
      layer 2: unit (j + 1) mod 19 sees unit j, minus 15 from the bias unit,
               so it fires (value 15) iff x_j = 1; unit 40 is a bias unit
               (b2 = 7.5); unit 41 sees unit 51 plus 15;
      layer 3: output i reads 2 x unit (i + 3) mod 19, plus 0.25 x unit 40,
               plus 0.125 x unit 41, plus b3_i = i / 8;
      then y = yt * out_std + out_mean."""
    W1 = np.zeros((19, 64)); b1 = np.zeros(64)
    W2 = np.zeros((64, 64)); b2 = np.zeros(64)
    W3 = np.zeros((64, 19)); b3 = np.arange(19) / 8.0
    for j in range(19):
        W1[j, j] = 30.0
        W2[j, (j + 1) % 19] = 1.0
        W2[63, (j + 1) % 19] = -0.5
    b1[63] = 30.0
    W1[1, 51], b1[51] = 30.0, -15.0
    W2[51, 41], b2[41] = 1.0, 15.0
    b2[40] = 7.5
    for i in range(19):
        W3[(i + 3) % 19, i] = 2.0
        W3[40, i] = 0.25
        W3[41, i] = 0.125
    in_mean = (np.arange(19) - 9) / 16.0
    in_std = np.where(np.arange(19) % 2 == 0, 2.0, 0.25)
    out_mean = np.full(19, -1.0)
    out_std = np.where(np.arange(19) % 3 == 0, 4.0, 0.5)
    p = mlp.Params(W1, b1, W2, b2, W3, b3, in_mean=in_mean, in_std=in_std, out_mean=out_mean,
                   out_std=out_std)
    v = np.array([1, -1, 0, 1, 1, 0, -1, 1, 0, 0, 1, -1, -1, 1, 0, 1, 0, 0, 1], np.float64)
    g = in_mean + in_std * v  # standardizes back to v exactly (powers of two)
    y = mlp.forward(p, g[None])[0]
    want = np.zeros(19)
    for i in range(19):
        s = (i + 3) % 19          # layer-2 unit read by output i ...
        j = (s - 1) % 19          # ... fires iff input j is +1
        unit = 15.0 if v[j] == 1 else 0.0
        unit41 = (15.0 if v[1] == 1 else 0.0) + 15.0
        yt = 2.0 * unit + 0.25 * 7.5 + 0.125 * unit41 + i / 8.0
        want[i] = yt * out_std[i] + out_mean[i]
    assert np.array_equal(y, want), (y, want)
