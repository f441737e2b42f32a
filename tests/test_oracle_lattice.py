"""Pins of the oracle's lattice-Boltzmann part against what the paper and the
mathematics fix (no GPU).  Each test names the passage it checks."""
import json
import os

import numpy as np
import pytest

import oracle
from helpers import oracle_sim
from paper_2210_06043_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_velocity_set_is_eq3():
    """Eq. (3): e_i = (cos((i-1)pi/2), sin((i-1)pi/2)) for i = 1..4 and
    sqrt(2)(cos((2i-9)pi/4), sin((2i-9)pi/4)) for i = 5..8."""
    ex, ey, w = oracle.lattice_tables()
    assert (ex[0], ey[0]) == (0, 0)
    for i in range(1, 5):
        a = (i - 1) * np.pi / 2
        assert (ex[i], ey[i]) == (round(np.cos(a)), round(np.sin(a)))
    for i in range(5, 9):
        a = (2 * i - 9) * np.pi / 4
        assert (ex[i], ey[i]) == (round(np.sqrt(2) * np.cos(a)), round(np.sqrt(2) * np.sin(a)))
    np.testing.assert_allclose(w, GOLD["d2q9_weights"]["value"], rtol=0, atol=1e-16)


def test_weight_moments_isotropy():
    """Lattice tensor identities of D2Q9 with c_s^2 = 1/3 (Sec. 2.1):
    sum w = 1, sum w e = 0, sum w e e = cs2 I, sum w e e e = 0,
    sum w e_a e_b e_c e_d = cs2^2 (d_ab d_cd + d_ac d_bd + d_ad d_bc)."""
    ex, ey, w = oracle.lattice_tables()
    e = np.stack([ex, ey], 1).astype(float)
    cs2 = GOLD["cs2"]["value"]
    assert abs(w.sum() - 1) < 1e-15
    np.testing.assert_allclose(w @ e, 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, e, e), cs2 * np.eye(2), atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", w, e, e, e), 0, atol=1e-16)
    d = np.eye(2)
    iso = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e), iso, atol=1e-16)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments(seed):
    """Eq. (2): the Hermite equilibrium has moments rho, rho u and
    rho (cs2 I + u u); stored shifted by w, h_eq = f_eq - w."""
    rng = np.random.default_rng(seed)
    ex, ey, w = oracle.lattice_tables()
    e = np.stack([ex, ey], 1).astype(float)
    drho = rng.uniform(-0.05, 0.05)
    u = rng.uniform(-0.08, 0.08, 2)
    h = oracle.heq(drho, *u)
    f = h + w
    rho = 1 + drho
    assert abs(f.sum() - rho) < 1e-15
    np.testing.assert_allclose(f @ e, rho * u, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", f, e, e), rho * (np.eye(2) / 3 + np.outer(u, u)),
                               atol=2e-16)


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_guo_moments(tau):
    """Eq. (4): sum F_i = 0, sum F_i e_i = (1 - 1/2tau) F,
    sum F_i e_i e_i = (1 - 1/2tau)(u F + F u)."""
    rng = np.random.default_rng(int(tau * 10))
    ex, ey, w = oracle.lattice_tables()
    e = np.stack([ex, ey], 1).astype(float)
    u = rng.uniform(-0.05, 0.05, 2)
    F = rng.uniform(-1e-3, 1e-3, 2)
    Fi = oracle.guo(tau, *u, *F)
    c = 1 - 1 / (2 * tau)
    assert abs(Fi.sum()) < 1e-18
    np.testing.assert_allclose(Fi @ e, c * F, rtol=1e-13, atol=1e-19)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", Fi, e, e), c * (np.outer(u, F) + np.outer(F, u)),
                               rtol=1e-12, atol=1e-19)


def _perturbed(cfg, seed, amp):
    """Oracle of ``cfg`` whose populations carry a seeded perturbation."""
    s = oracle_sim(cfg)
    A = s.populations()
    rng = np.random.default_rng(seed)
    A = A + amp * rng.standard_normal(A.shape)
    s.set_populations(A)
    return s


@pytest.mark.parametrize("walls", [0, 3])
def test_mass_conserved(walls):
    """Bounce-back and periodic streaming move populations without loss, the
    BGK collision keeps rho and sum F_i = 0 (Eqs. 1, 2, 4): sum of drho is
    constant to round-off, also with a body and its spread force."""
    cfg = inputs.config_tiny(walls=walls)
    s = _perturbed(cfg, 11, 1e-4)
    m0 = s.totals()[0]
    s.step(150)
    m1 = s.totals()[0]
    assert abs(m1 - m0) < 1e-15 * 9 * cfg.nx * cfg.ny


def _steady_channel(ny, tau, g, steps):
    s = oracle.Sim(2, ny, tau, g, 0.0, 3)
    s.init_flow(None)
    s.step(steps)
    return s


@pytest.mark.parametrize("tau", [1.0, 0.5 + np.sqrt(3.0 / 16.0), 1.5])
def test_poiseuille_closed_form(tau):
    """Body-force driven channel between halfway bounce-back walls at
    y = -1/2 and y = H - 1/2, started from rest.  The steady discrete
    solution of BGK with Guo forcing is the parabola u = g/(2 nu) eta (H - eta),
    eta = y + 1/2, plus a uniform slip g (16 L - 3)/(24 nu), L = (tau - 1/2)^2
    (the slip vanishes at L = 3/16); drho = 0."""
    H, g = 20, 1e-6
    nu = (tau - 0.5) / 3
    s = _steady_channel(H, tau, g, 14000)
    drho, ux, uy = s.macro()
    eta = np.arange(H) + 0.5
    lam = (tau - 0.5) ** 2
    exact = g / (2 * nu) * eta * (H - eta) + g * (16 * lam - 3) / (24 * nu)
    umax = exact.max()
    assert np.abs(ux - exact[:, None]).max() < 1e-12 * umax
    assert np.abs(uy).max() < 1e-13 * umax
    assert np.abs(drho).max() < 1e-16


def test_poiseuille_stress_closed_form():
    """At the steady channel flow, the viscous stress from the
    non-equilibrium populations, -(1 - 1/2tau) Pi_neq_xy, equals
    rho nu du/dy = g (H - 2 eta)/2 exactly (Sec. 2.6 reading of Eq. 15)."""
    H, g, tau = 20, 1e-6, 1.0
    s = _steady_channel(H, tau, g, 14000)
    s.step(1)
    f = s.node_fields()
    eta = np.arange(H) + 0.5
    exact = g * (H - 2 * eta) / 2
    np.testing.assert_allclose(f["sxy"][:, 0], exact, rtol=1e-9, atol=1e-12 * g * H)
    # the normal components carry only the O(u F) forcing imprint of Pi_neq
    _, ux, _ = s.macro()
    assert np.abs(f["sxx"]).max() < 4 * np.abs(ux).max() * g
    assert np.abs(f["syy"]).max() < 4 * np.abs(ux).max() * g


def test_momentum_balance_periodic():
    """Fully periodic box: BGK with Guo forcing adds exactly F per node to the
    post-collision momentum, streaming only moves it, so the total momentum
    of the stored populations grows by N g + sum f_ib per step, and the spread
    force totals sum_v dV_v (U_v - u*_v) (the renormalised weights sum to 1)."""
    cfg = inputs.config_tiny(walls=0)
    cfg.gx, cfg.gy = 2e-6, -1e-6
    s = _perturbed(cfg, 5, 1e-5)
    s.step(20)
    for _ in range(3):
        p0 = s.totals()[1:]
        xs = [s.vertices(k).copy() for k in range(len(cfg.bodies))]
        s.step(1)
        p1 = s.totals()[1:]
        f = s.node_fields()
        N = cfg.nx * cfg.ny
        expect = np.array([N * cfg.gx + f["fibx"].sum(), N * cfg.gy + f["fiby"].sum()])
        np.testing.assert_allclose(p1 - p0, expect, rtol=1e-10, atol=1e-18)
        lag = np.zeros(2)
        for k in range(len(cfg.bodies)):
            w = s.body_work(k)
            x = xs[k]
            seg = np.hypot(*(np.roll(x, -1, 0) - x).T)
            dV = 0.5 * (seg + np.roll(seg, 1))
            lag += (dV[:, None] * (w["U"] - w["ustar"])).sum(0)
        np.testing.assert_allclose([f["fibx"].sum(), f["fiby"].sum()], lag, rtol=1e-11, atol=1e-20)


def test_init_flow_is_equilibrium():
    """The initial populations are h_eq(drho = 0, u_P(y)) (Sec. 3.1, flow
    established before the cell is released): the macroscopic velocity read
    back equals the prescribed profile up to the g/2 half-force shift."""
    cfg = inputs.lattice_only(5, 12, 0.9)
    s = oracle_sim(cfg)
    A = s.populations()
    ex, ey, w = oracle.lattice_tables()
    jx = np.einsum("q,qyx->yx", ex.astype(float), A)
    np.testing.assert_allclose(jx[:, 0], cfg.ux_init, rtol=1e-13)
