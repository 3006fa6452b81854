"""Pins of the D3Q27 build of the FP64 oracle (the lattice of the paper's
block-sparse register study), against facts fixed by the mathematics:
exact rational lattice identities (isotropy through fourth order and the
sixth-order corner moment), equilibrium moments, fixed points, the
regularized operator in Hermite space, Taylor-Green decay, Couette flow,
mass conservation with obstacles and with the moving lid, and a brute-force
numpy restatement of a periodic step with solids."""
from fractions import Fraction
import math

import numpy as np
import pytest

from paper_2503_07898_amd import workloads

Q27 = 27


def _rational(w):
    out = [Fraction(x).limit_denominator(1000) for x in w]
    for a, b in zip(out, w):
        assert abs(float(a) - b) < 1e-16
    return out


def test_lattice_rational_moments_d3q27(orc):
    c, w, opp = orc.lattice(Q27)
    W = _rational(w)
    cs2 = Fraction(1, 3)
    assert sum(W) == 1
    d = lambda a, b: 1 if a == b else 0
    for a in range(3):
        assert sum(W[i] * c[i, a] for i in range(Q27)) == 0
        for b in range(3):
            assert sum(W[i] * c[i, a] * c[i, b] for i in range(Q27)) == cs2 * d(a, b)
            for g in range(3):
                assert sum(W[i] * c[i, a] * c[i, b] * c[i, g] for i in range(Q27)) == 0
                for e in range(3):
                    m4 = sum(W[i] * c[i, a] * c[i, b] * c[i, g] * c[i, e] for i in range(Q27))
                    # D3Q27 is isotropic to fourth order, diagonal included
                    assert m4 == cs2 * cs2 * (d(a, b) * d(g, e) + d(a, g) * d(b, e) + d(a, e) * d(b, g))
    # sixth-order moment carried by the corners: sum w cx^2 cy^2 cz^2 = cs^6
    assert sum(W[i] * c[i, 0] ** 2 * c[i, 1] ** 2 * c[i, 2] ** 2 for i in range(Q27)) == cs2 ** 3
    assert len({tuple(v) for v in c}) == Q27
    for i in range(Q27):
        assert (c[opp[i]] == -c[i]).all()
    assert (np.abs(c).sum(1) == [0] + [1] * 6 + [2] * 12 + [3] * 8).all()
    # the first 19 directions are the D3Q19 ones, in the same order
    c19, _, _ = orc.lattice(19)
    assert np.array_equal(c[:19], c19)


def test_equilibrium_moments_and_fixed_points_d3q27(orc):
    c, w, _ = orc.lattice(Q27)
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.8, 1.2)
        u = rng.uniform(-0.1, 0.1, 3)
        feq = orc.equilibrium(rho, u, Q27)
        assert abs(feq.sum() - rho) < 1e-15
        assert np.allclose(c.T @ feq, rho * u, atol=1e-16, rtol=0)
        P = np.einsum("ia,ib,i->ab", c, c, feq)
        assert np.allclose(P, rho / 3 * np.eye(3) + rho * np.outer(u, u), atol=1e-15, rtol=0)
        for tau in (0.5038, 0.6, 1.3):
            assert np.max(np.abs(orc.collide_bgk(feq, tau) - feq)) <= 2e-15
            assert np.max(np.abs(orc.collide_regularized(feq, tau) - feq)) <= 2e-15


def test_regularized_in_hermite_space_d3q27(orc):
    c, w, _ = orc.lattice(Q27)
    rng = np.random.default_rng(3)
    for _ in range(10):
        f = orc.equilibrium(rng.uniform(0.9, 1.1), rng.uniform(-0.08, 0.08, 3), Q27)
        f = f * (1 + 0.05 * rng.standard_normal(Q27))
        tau = rng.uniform(0.51, 1.5)
        out = orc.collide_regularized(f, tau)
        assert abs(out.sum() - f.sum()) < 1e-15
        assert np.allclose(c.T @ out, c.T @ f, atol=1e-16, rtol=0)
        rho, u = orc.moments(f)
        feq = orc.equilibrium(rho, u, Q27)
        A = rng.standard_normal((3, 3)) * 1e-3
        Pi = A + A.T
        Qi = np.einsum("ia,ib->iab", c, c) - np.eye(3)[None] / 3
        f1 = w * 4.5 * np.einsum("iab,ab->i", Qi, Pi)
        g = feq + f1
        assert np.allclose(orc.collide_regularized(g, tau), orc.collide_bgk(g, tau), atol=1e-15, rtol=0)
        assert np.allclose(orc.f1_projection(g, feq), f1, atol=1e-16, rtol=0)


def test_taylor_green_decay_d3q27(orc):
    n, u0, tau, steps = 32, 0.05, 0.6, 100
    k = 2 * math.pi / n
    nu = (tau - 0.5) / 3
    rho0, u_init = workloads.taylor_green_2d(n, u0)
    g = orc.Grid(n, n, n, tau=tau, q=Q27)
    f = g.run(g.init_equilibrium(rho0, u_init), steps)
    _, u = g.macroscopic(f)
    expect = u_init * math.exp(-2 * nu * k * k * steps)
    assert orc.rel_l2(u, expect) < 1e-2


def _numpy_periodic_step(f, fluid, tau, c, w, opp):
    g = np.empty_like(f)
    for i in range(len(w)):
        shift = (int(c[i, 2]), int(c[i, 1]), int(c[i, 0]))
        pulled = np.roll(f[..., i], shift, axis=(0, 1, 2))
        src_fluid = np.roll(fluid, shift, axis=(0, 1, 2))
        g[..., i] = np.where(src_fluid, pulled, f[..., opp[i]])
    rho = g.sum(-1)
    u = np.einsum("zyxi,ia->zyxa", g, c) / rho[..., None]
    cu = np.einsum("zyxa,ia->zyxi", u, c)
    uu = (u * u).sum(-1)[..., None]
    feq = w * rho[..., None] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
    out = g - (g - feq) / tau
    out[~fluid] = 0
    return out


def test_bruteforce_numpy_periodic_with_solids_d3q27(orc):
    c, w, opp = orc.lattice(Q27)
    n = (10, 9, 8)
    rng = np.random.default_rng(5)
    fluid = rng.random((n[2], n[1], n[0])) > 0.25
    g = orc.Grid(*n, fluid=fluid.astype(np.uint8), tau=0.7, q=Q27)
    f = g.init_equilibrium(1 + 0.02 * rng.standard_normal(fluid.shape),
                           0.04 * rng.standard_normal(fluid.shape + (3,)))
    f[~fluid] = 0
    a, b = f.copy(), f.copy()
    for _ in range(5):
        a = g.step(a)
        a[~fluid] = 0
        b = _numpy_periodic_step(b, fluid, 0.7, c, w, opp)
    assert np.max(np.abs(a - b)) < 1e-14


def test_walls_conserve_mass_d3q27(orc):
    n = 12
    fluid = workloads.random_mask(n, n, n, seed=11, solid_fraction=0.2, empty_block_fraction=0.1)
    g = orc.Grid(n, n, n, fluid=fluid, tau=0.58, q=Q27)
    f = g.init_equilibrium(1.0, np.array([0.05, 0.01, -0.02]))
    f[fluid == 0] = 0
    m0 = f.sum()
    f = g.run(f, 100)
    f[fluid == 0] = 0
    assert abs(f.sum() - m0) / m0 < 1e-13
    # closed cavity with the lid winning at edges and corners: the corner
    # links' lid terms cancel in pairs as the edge links' do
    bc = [(orc.BB, (0, 0, 0))] * 5 + [(orc.MOVING, (0.1, 0.0, 0.0))]
    g = orc.Grid(n, n, n, periodic=(False, False, False), bc=bc, tau=0.55, q=Q27)
    f = g.init_equilibrium(1.0, np.zeros(3))
    m0 = f.sum()
    f = g.run(f, 200)
    assert abs(f.sum() - m0) / m0 < 1e-13
    _, u = g.macroscopic(f)
    assert u[-1, :, :, 0].mean() > 0.01


def test_couette_linear_profile_d3q27(orc):
    H, uw = 16, 0.05
    bc = [(orc.BB, (0, 0, 0))] * 6
    bc[orc.YMAX] = (orc.MOVING, (uw, 0.0, 0.0))
    g = orc.Grid(1, H, 1, periodic=(True, False, True), bc=bc, tau=1.0, q=Q27)
    f = g.run(g.init_equilibrium(1.0, np.zeros(3)), 8000)
    _, u = g.macroscopic(f)
    assert orc.rel_l2(u[0, :, 0, 0], uw * (np.arange(H) + 0.5) / H) < 1e-6


@pytest.mark.parametrize("seed", [0, 1])
def test_reference_builder_d3q27_neighbours(orc, seed):
    n = (12, 8, 16)
    periodic = (seed == 0, True, False)
    fluid = workloads.random_mask(*n, seed=200 + seed, empty_block_fraction=0.3)
    ref = orc.build_block_maps(*n, periodic, fluid, [orc.BB] * 6, False, q=Q27)
    c, _, _ = orc.lattice(Q27)
    nb = len(ref["coords"])
    pos = {tuple(v): s for s, v in enumerate(ref["coords"])}
    nba = (n[0] // 4, n[1] // 4, n[2] // 4)
    assert ref["nbr"].shape == (nb, 26)
    for s in range(nb):
        for d in range(1, Q27):
            t = [int(ref["coords"][s, a]) + int(c[d, a]) for a in range(3)]
            ok = all(periodic[a] or 0 <= t[a] < nba[a] for a in range(3))
            t = tuple(t[a] % nba[a] for a in range(3))
            assert ref["nbr"][s, d - 1] == (pos.get(t, -1) if ok else -1)
