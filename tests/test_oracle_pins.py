"""Pins of the FP64 oracle against facts fixed by the mathematics.

Each test checks the oracle against something other than itself: exact
rational lattice identities, closed-form flow solutions (Taylor-Green decay,
Couette, Poiseuille), exact invariants (mass conservation, translation
equivariance, fixed points) and a brute-force numpy restatement on tiny
periodic boxes.  None of them calls the GPU library.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

from paper_2503_07898_amd import workloads


# ---------------------------------------------------------------- lattice ---

def _rational_weights(w):
    out = [Fraction(x).limit_denominator(1000) for x in w]
    for a, b in zip(out, w):
        assert abs(float(a) - b) < 1e-16
    return out


def test_lattice_rational_moments(orc):
    """D3Q19 isotropy: sum w = 1, sum w c = 0, sum w c_a c_b = cs2 delta,
    odd third moment 0, fourth moment cs4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)."""
    c, w, opp = orc.lattice()
    W = _rational_weights(w)
    cs2 = Fraction(1, 3)
    assert sum(W) == 1
    d = lambda a, b: 1 if a == b else 0
    for a in range(3):
        assert sum(W[i] * c[i, a] for i in range(19)) == 0
        for b in range(3):
            assert sum(W[i] * c[i, a] * c[i, b] for i in range(19)) == cs2 * d(a, b)
            for g in range(3):
                assert sum(W[i] * c[i, a] * c[i, b] * c[i, g] for i in range(19)) == 0
                for e in range(3):
                    m4 = sum(W[i] * c[i, a] * c[i, b] * c[i, g] * c[i, e] for i in range(19))
                    iso = cs2 * cs2 * (d(a, b) * d(g, e) + d(a, g) * d(b, e) + d(a, e) * d(b, g))
                    # D3Q19 is isotropic to fourth order except the c_a^4 diagonal
                    if a == b == g == e:
                        assert m4 == Fraction(1, 3)
                    else:
                        assert m4 == iso
    # 19 distinct velocities, opposite pairs, rest first, 6 faces then 12 edges
    assert len({tuple(v) for v in c}) == 19
    for i in range(19):
        assert (c[opp[i]] == -c[i]).all()
    assert (np.abs(c).sum(1) == [0] + [1] * 6 + [2] * 12).all()


def test_equilibrium_moments(orc):
    c, w, _ = orc.lattice()
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.8, 1.2)
        u = rng.uniform(-0.1, 0.1, 3)
        feq = orc.equilibrium(rho, u)
        assert abs(feq.sum() - rho) < 1e-15
        assert np.allclose(c.T @ feq, rho * u, atol=1e-16, rtol=0)
        P = np.einsum("ia,ib,i->ab", c, c, feq)
        assert np.allclose(P, rho / 3 * np.eye(3) + rho * np.outer(u, u), atol=1e-15, rtol=0)


@pytest.mark.parametrize("collide", ["bgk", "regularized"])
def test_equilibrium_is_fixed_point(orc, collide):
    rng = np.random.default_rng(2)
    op = orc.collide_bgk if collide == "bgk" else orc.collide_regularized
    for tau in (0.503820, 0.55, 0.6, 1.0, 1.7):
        rho = rng.uniform(0.9, 1.1)
        u = rng.uniform(-0.1, 0.1, 3)
        feq = orc.equilibrium(rho, u)
        assert np.max(np.abs(op(feq, tau) - feq)) <= 1e-15 * 2


def test_regularized_conserves_and_matches_bgk_in_hermite_space(orc):
    c, w, _ = orc.lattice()
    rng = np.random.default_rng(3)
    for _ in range(20):
        f = orc.equilibrium(rng.uniform(0.9, 1.1), rng.uniform(-0.08, 0.08, 3))
        f = f * (1 + 0.05 * rng.standard_normal(19))
        tau = rng.uniform(0.51, 1.5)
        out = orc.collide_regularized(f, tau)
        assert abs(out.sum() - f.sum()) < 1e-15
        assert np.allclose(c.T @ out, c.T @ f, atol=1e-16, rtol=0)
        # f = f^eq + f1(Pi) for a random symmetric traceful Pi: both operators agree
        rho, u = orc.moments(f)
        feq = orc.equilibrium(rho, u)
        A = rng.standard_normal((3, 3)) * 1e-3
        Pi = A + A.T
        Qi = np.einsum("ia,ib->iab", c, c) - np.eye(3)[None] / 3
        f1 = w * 4.5 * np.einsum("iab,ab->i", Qi, Pi)
        g = feq + f1
        assert np.allclose(orc.collide_regularized(g, tau), orc.collide_bgk(g, tau), atol=1e-15, rtol=0)
        # and the projection returns f1 itself
        assert np.allclose(orc.f1_projection(g, feq), f1, atol=1e-16, rtol=0)


# ------------------------------------------------------------ dense flows ---

def test_taylor_green_decay_32(orc):
    """2D Taylor-Green vortex extruded in z, 32^3 periodic, tau = 0.6, 100 steps:
    u(t) = u(0) exp(-2 nu k^2 t) with nu = (tau - 1/2)/3."""
    n, u0, tau, steps = 32, 0.05, 0.6, 100
    k = 2 * math.pi / n
    nu = (tau - 0.5) / 3
    rho0, u_init = workloads.taylor_green_2d(n, u0)
    g = orc.Grid(n, n, n, tau=tau)
    f = g.init_equilibrium(rho0, u_init)
    energies = []
    for s in range(0, steps, 10):
        rho, u = g.macroscopic(f)
        energies.append(0.5 * np.sum(rho * (u ** 2).sum(-1)))
        f = g.run(f, 10)
    rho, u = g.macroscopic(f)
    energies.append(0.5 * np.sum(rho * (u ** 2).sum(-1)))
    expect = u_init * math.exp(-2 * nu * k * k * steps)
    err = orc.rel_l2(u, expect)
    assert err < 1e-2, err
    t = np.arange(len(energies)) * 10.0
    rate = -np.polyfit(t[2:], np.log(energies[2:]), 1)[0]
    assert abs(rate / (4 * nu * k * k) - 1) < 0.02, rate / (4 * nu * k * k)


def test_uniform_flow_fixed_point_periodic(orc):
    g = orc.Grid(8, 6, 5, tau=0.55)
    f = g.init_equilibrium(1.0, np.array([0.04, -0.02, 0.01]))
    out = g.run(f, 10)
    assert np.max(np.abs(out - f)) <= 1e-15


def test_translation_equivariance(orc):
    n = 12
    rng = np.random.default_rng(4)
    rho = 1 + 0.01 * rng.standard_normal((n, n, n))
    u = 0.03 * rng.standard_normal((n, n, n, 3))
    for coll in (orc.BGK, orc.REGULARIZED):
        g = orc.Grid(n, n, n, tau=0.57, collision=coll)
        f = g.init_equilibrium(rho, u)
        a = g.run(f, 7)
        for axis in (0, 1, 2):
            fs = np.roll(f, 1, axis=axis)
            b = g.run(fs, 7)
            assert np.array_equal(np.roll(a, 1, axis=axis), b)


def _numpy_periodic_step(f, fluid, tau, c, w, opp):
    """Brute-force restatement: periodic box, halfway bounce-back on solid
    voxels, BGK.  f is (nz,ny,nx,19) post-collision; returns the next one."""
    g = np.empty_like(f)
    for i in range(19):
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


def test_bruteforce_numpy_periodic_with_solids(orc):
    c, w, opp = orc.lattice()
    n = (10, 9, 8)
    rng = np.random.default_rng(5)
    fluid = (rng.random((n[2], n[1], n[0])) > 0.25)
    g = orc.Grid(*n, fluid=fluid.astype(np.uint8), tau=0.7)
    rho = 1 + 0.02 * rng.standard_normal(fluid.shape)
    u = 0.04 * rng.standard_normal(fluid.shape + (3,))
    f = g.init_equilibrium(rho, u)
    f[~fluid] = 0
    a = f.copy()
    b = f.copy()
    for _ in range(5):
        a = g.step(a)
        a[~fluid] = 0
        b = _numpy_periodic_step(b, fluid, 0.7, c, w, opp)
    assert np.max(np.abs(a - b)) < 1e-14


def test_all_fluid_mask_equals_no_mask(orc):
    n = 8
    rho, u = workloads.taylor_green_2d(n, 0.05)
    g0 = orc.Grid(n, n, n, tau=0.6)
    g1 = orc.Grid(n, n, n, tau=0.6, fluid=np.ones((n, n, n), np.uint8))
    f = g0.init_equilibrium(rho, u)
    assert np.array_equal(g0.run(f, 5), g1.run(f, 5))


# ---------------------------------------------------------- walls and BCs ---

def test_obstacles_conserve_mass(orc):
    n = 16
    fluid = workloads.random_mask(n, n, n, seed=11, solid_fraction=0.2, empty_block_fraction=0.1)
    g = orc.Grid(n, n, n, fluid=fluid, tau=0.58)
    f = g.init_equilibrium(1.0, np.array([0.05, 0.01, -0.02]))
    f[fluid == 0] = 0
    m0 = f.sum()
    f = g.run(f, 200)
    f[fluid == 0] = 0
    assert abs(f.sum() - m0) / m0 < 1e-13


def test_cavity_lid_conserves_mass(orc):
    """Closed cavity, moving lid at z max: the moving-wall terms cancel in
    pairs when the lid wins at edges, so total mass is exact."""
    n = 12
    bc = [(orc.BB, (0, 0, 0))] * 5 + [(orc.MOVING, (0.1, 0.0, 0.0))]
    g = orc.Grid(n, n, n, periodic=(False, False, False), bc=bc, tau=0.55)
    f = g.init_equilibrium(1.0, np.zeros(3))
    m0 = f.sum()
    f = g.run(f, 400)
    assert abs(f.sum() - m0) / m0 < 1e-13
    rho, u = g.macroscopic(f)
    assert u[-1, :, :, 0].mean() > 0.01  # the lid drives the top layer


def test_couette_linear_profile(orc):
    H, uw = 16, 0.05
    bc = [(orc.BB, (0, 0, 0))] * 6
    bc[orc.YMAX] = (orc.MOVING, (uw, 0.0, 0.0))
    g = orc.Grid(1, H, 1, periodic=(True, False, True), bc=bc, tau=1.0)
    f = g.init_equilibrium(1.0, np.zeros(3))
    f = g.run(f, 8000)
    _, u = g.macroscopic(f)
    y = np.arange(H)
    expect = uw * (y + 0.5) / H
    assert orc.rel_l2(u[0, :, 0, 0], expect) < 1e-6


def test_regularized_uniform_flow_fixed_point(orc):
    u0 = np.array([0.05, 0.0, 0.0])
    bc = [(orc.BB, (0, 0, 0))] * 6
    bc[orc.XMIN] = (orc.REG_VEL, tuple(u0))
    bc[orc.XMAX] = (orc.REG_PRES, (1.0, 0, 0))
    for coll in (orc.BGK, orc.REGULARIZED):
        g = orc.Grid(12, 4, 4, periodic=(False, True, True), bc=bc, tau=0.6, collision=coll)
        f = g.init_equilibrium(1.0, u0)
        out = g.run(f, 10)
        assert np.max(np.abs(out - f)) < 1e-15


def _poiseuille_error(orc, H):
    nx = 4 * H
    drho = 5e-4 * 16 / H
    bc = [(orc.BB, (0, 0, 0))] * 6
    bc[orc.XMIN] = (orc.REG_PRES, (1.0 + drho, 0, 0))
    bc[orc.XMAX] = (orc.REG_PRES, (1.0 - drho, 0, 0))
    tau = 0.8
    nu = (tau - 0.5) / 3
    g = orc.Grid(nx, H, 1, periodic=(False, False, True), bc=bc, tau=tau)
    f = g.init_equilibrium(1.0, np.zeros(3))
    f = g.run(f, int(12 * H * H / (nu * math.pi ** 2)))
    rho, u = g.macroscopic(f)
    xm = nx // 2
    grad = (rho[0, :, xm + 1].mean() - rho[0, :, xm - 1].mean()) / 2.0
    G = -grad / 3.0
    rbar = rho[0, :, xm].mean()
    y = np.arange(H)
    expect = G / (2 * rbar * nu) * (y + 0.5) * (H - 0.5 - y)
    # the regularized pressure faces impose zero tangential velocity
    assert np.max(np.abs(u[0, :, 0, 1])) < 1e-15
    assert np.max(np.abs(rho[0, :, 0] - (1 + drho))) < 1e-15
    return orc.rel_l2(u[0, :, xm, 0], expect)


@pytest.mark.slow
def test_poiseuille_pressure_driven(orc):
    e16 = _poiseuille_error(orc, 16)
    e32 = _poiseuille_error(orc, 32)
    assert e16 < 1e-2 and e32 < 1e-2, (e16, e32)
    assert e16 / e32 > 2.5, (e16, e32)  # close to second order in 1/H


def test_velocity_inlet_develops_parabola(orc):
    """Plug inflow through a regularized velocity face between two walls
    develops a parabolic profile carrying the same flux."""
    H, nx, u0 = 12, 72, 0.03
    bc = [(orc.BB, (0, 0, 0))] * 6
    bc[orc.XMIN] = (orc.REG_VEL, (u0, 0, 0))
    bc[orc.XMAX] = (orc.REG_PRES, (1.0, 0, 0))
    tau = 0.8
    nu = (tau - 0.5) / 3
    g = orc.Grid(nx, H, 1, periodic=(False, False, True), bc=bc, tau=tau)
    f = g.init_equilibrium(1.0, np.array([u0, 0, 0]))
    f = g.run(f, int(14 * H * H / (nu * math.pi ** 2)))
    rho, u = g.macroscopic(f)
    assert np.max(np.abs(u[0, :, 0, :] - [u0, 0, 0])) < 1e-15  # imposed exactly
    xm = nx // 2
    y = np.arange(H)
    shape = (y + 0.5) * (H - 0.5 - y)
    prof = u[0, :, xm, 0]
    coef = prof @ shape / (shape @ shape)
    assert orc.rel_l2(prof, coef * shape) < 1e-2
    # steady mass flux rho*u_x summed over a cross-section is the same at the
    # inlet (where u = u0 exactly and rho is solved for) and downstream
    flux = (rho[0] * u[0, :, :, 0]).sum(0)
    assert np.max(np.abs(flux[: nx // 2] / flux[0] - 1)) < 1e-4
