"""Pins of the FP64 oracle of the 3D extension's lattice (D3Q19 BGK with the
Guo term, halfway bounce-back walls): lattice isotropy, equilibrium and
forcing moments, exact conservation, the closed-form steady profile between
two walls, and the tube's symmetry and Hagen-Poiseuille flow rate."""

import numpy as np
import pytest

from oracle import tube3d


def test_d3q19_tables_are_isotropic_to_fourth_order():
    """Sum w = 1; odd moments vanish; sum w e_a e_b = delta/3; sum w e_a e_b e_c
    e_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc)/9: the conditions under which
    the equilibrium of Eq. (2) recovers Navier-Stokes with c_s^2 = 1/3."""
    e, w = tube3d.lattice_tables()
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    d = np.eye(3)
    for a in range(3):
        assert abs(np.sum(w * e[:, a])) < 1e-15
        for b in range(3):
            assert np.sum(w * e[:, a] * e[:, b]) == pytest.approx(d[a, b] / 3, abs=1e-15)
            for c in range(3):
                assert abs(np.sum(w * e[:, a] * e[:, b] * e[:, c])) < 1e-15
                for g in range(3):
                    want = (d[a, b] * d[c, g] + d[a, c] * d[b, g] + d[a, g] * d[b, c]) / 9
                    assert np.sum(w * e[:, a] * e[:, b] * e[:, c] * e[:, g]) == pytest.approx(want, abs=1e-15)
    # the 19 velocities: rest, 6 axis directions, 12 face diagonals, no repeats,
    # every one with its opposite
    norms = sorted(int(v @ v) for v in e)
    assert norms == [0] + [1] * 6 + [2] * 12
    assert len({tuple(v) for v in e}) == 19
    assert all(tuple(-v) in {tuple(u) for u in e} for v in e)


@pytest.mark.parametrize("drho,u", [(0.0, (0.0, 0.0, 0.0)), (2e-3, (3e-3, -1e-3, 2e-3)), (-1e-2, (0.02, 0.01, -0.015))])
def test_equilibrium_moments(drho, u):
    """Eq. (2): sum f_eq = rho, sum f_eq e = rho u, sum f_eq e e = rho/3 I + rho u u
    (shifted by w: the zeroth moment is drho, the second rho/3 I + rho u u - I/3)."""
    e, w = tube3d.lattice_tables()
    h = tube3d.heq(drho, *u)
    rho = 1.0 + drho
    u = np.array(u)
    assert h.sum() == pytest.approx(drho, abs=1e-15)
    np.testing.assert_allclose(e.T @ h, rho * u, rtol=0, atol=1e-15)
    P = (e.T * h) @ e
    np.testing.assert_allclose(P, rho / 3 * np.eye(3) + rho * np.outer(u, u) - np.eye(3) / 3, rtol=0, atol=1e-15)


def test_guo_moments():
    """Eq. (4): sum F_i = 0, sum F_i e = (1 - 1/(2 tau)) F, sum F_i e e =
    (1 - 1/(2 tau)) (u F + F u)."""
    e, _ = tube3d.lattice_tables()
    tau, u, F = 0.8, np.array([0.01, -0.004, 0.002]), np.array([2e-5, 1e-5, -3e-5])
    Fi = tube3d.guo(tau, u, F)
    c = 1 - 0.5 / tau
    assert abs(Fi.sum()) < 1e-20
    np.testing.assert_allclose(e.T @ Fi, c * F, rtol=0, atol=1e-20)
    np.testing.assert_allclose((e.T * Fi) @ e, c * (np.outer(u, F) + np.outer(F, u)), rtol=0, atol=1e-20)


def _random_state(t, rng, amp=1e-4):
    A = t.populations()
    fl = t.fluid()
    A += amp * rng.standard_normal(A.shape) * fl[None, :, :, None]
    t.set_populations(A)


@pytest.mark.parametrize("tau", [1.0, 0.7])
def test_mass_conserved_and_momentum_grows_by_the_body_force(tau):
    """Streaming, bounce-back and the collision conserve mass exactly; in a
    periodic box each step adds g to the stored momentum of every node (the
    Guo term with u taken at half the force)."""
    rng = np.random.default_rng(3)
    t = tube3d.Tube(10, 12, 12, tau, 0.0, radius=5.5)
    t.init_flow()
    _random_state(t, rng)
    m0 = t.totals()[0]
    t.step(50)
    assert abs(t.totals()[0] - m0) < 1e-14 * t.fluid().sum() * 10
    g = 2e-6
    b = tube3d.Tube(6, 5, 7, tau, g, geom=tube3d.BOX)
    b.init_flow()
    _random_state(b, rng)
    p0 = b.totals()
    b.step(20)
    p1 = b.totals()
    N = 6 * 5 * 7
    assert p1[1] - p0[1] == pytest.approx(20 * N * g, rel=1e-9)
    assert abs(p1[2] - p0[2]) < 1e-15 and abs(p1[3] - p0[3]) < 1e-15
    assert abs(p1[0] - p0[0]) < 1e-13


@pytest.mark.parametrize("tau", [1.0, 0.8])
def test_slab_poiseuille_closed_form(tau):
    """Between two halfway bounce-back walls (fluid rows z = 0 .. H-1) the
    steady BGK solution with the Guo term is u(z) = g/(2 nu) eta (H - eta) +
    g (16 L - 3)/(24 nu), eta = z + 1/2, L = (tau - 1/2)^2: the x-momentum
    exchange across the walls involves only the four x-z face diagonals of
    D3Q19, the same sub-lattice as D2Q9's diagonals, so the discrete solution
    of the 2D channel holds for the slab."""
    H, g = 8, 1e-6
    nu = (tau - 0.5) / 3
    t = tube3d.Tube(2, 2, H, tau, g, geom=tube3d.SLAB)
    t.init_flow()
    t.step(6000)
    _, ux, uy, uz = t.macro()
    eta = np.arange(H) + 0.5
    Lam = (tau - 0.5) ** 2
    want = g / (2 * nu) * eta * (H - eta) + g * (16 * Lam - 3) / (24 * nu)
    np.testing.assert_allclose(ux[:, 0, 0], want, rtol=1e-9, atol=0)
    assert np.abs(uy).max() < 1e-18 and np.abs(uz).max() < 1e-18


def test_tube_symmetry_and_hagen_poiseuille_rate():
    """The staircase tube is symmetric under y <-> z and reflections of y and
    z, so is its flow; its steady flow rate is Hagen-Poiseuille's, pi g R^4 /
    (8 nu), for the radius of the circle with the tube's cross-section area
    (fluid nodes / pi), up to the staircase wall: 1.8 % below at R = 8 and
    at R = 12 alike."""
    R, g, tau = 8.0, 1e-7, 1.0
    nu = (tau - 0.5) / 3
    n = 18
    t = tube3d.Tube(2, n, n, tau, g, radius=R)
    fl = t.fluid()
    yy, zz = np.meshgrid(np.arange(n) - (n - 1) / 2, np.arange(n) - (n - 1) / 2)
    prof = np.where(fl, g / (4 * nu) * np.maximum(R * R - yy ** 2 - zz ** 2, 0.0), 0.0)
    t.init_flow(prof)
    t.step(4000)
    _, ux, _, _ = t.macro()
    u = ux[:, :, 0]
    np.testing.assert_allclose(u, u.T, rtol=0, atol=1e-15 * np.abs(u).max())
    np.testing.assert_allclose(u, u[::-1, :], rtol=0, atol=1e-15 * np.abs(u).max())
    np.testing.assert_allclose(u, u[:, ::-1], rtol=0, atol=1e-15 * np.abs(u).max())
    q = u.sum()
    r_area = np.sqrt(fl.sum() / np.pi)
    q_hp = np.pi * g * r_area ** 4 / (8 * nu)
    assert abs(q / q_hp - 1) < 0.03, q / q_hp


# ---- fixed immersed bodies: cosine-delta interpolation and spreading in 3D ----------

from paper_2210_06043_amd import inputs  # noqa: E402  (geometry generator, no method arithmetic)


def test_vertex_weights_are_the_surface_area():
    """Each vertex carries a third of its triangles' area: the weights sum to
    the triangulated surface area, within 0.5 % of 4 pi R^2 at level 3."""
    xyz, tri = inputs.icosphere(3, 4.0, (8.0, 8.5, 8.5))
    t = tube3d.Tube(16, 17, 17, 1.0, 0.0, geom=tube3d.BOX)
    t.add_fixed_body(xyz, tri)
    w = t.vertex_weights()
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1).sum()
    assert w.sum() == pytest.approx(area, rel=1e-12)
    assert abs(area / (4 * np.pi * 16.0) - 1) < 0.005


def test_uniform_flow_is_interpolated_exactly_and_spread_force_totals_the_body_force():
    """The 4-point cosine delta sums to one over the nodes of any stencil, so a
    uniform flow U interpolates to U at every vertex; with U = 0 on the
    body the direct force is -U dV per vertex and the spread field's total
    is -U times the surface area; one step then changes the stored momentum
    by exactly that total (periodic box, no drive)."""
    U = np.array([2e-4, -1e-4, 5e-5])
    t = tube3d.Tube(16, 17, 18, 0.9, 0.0, geom=tube3d.BOX)
    xyz, tri = inputs.icosphere(3, 3.5, (7.3, 8.1, 8.7))
    t.add_fixed_body(xyz, tri)
    A = t.populations()
    heq = tube3d.heq(0.0, *U)
    A[:] = heq[:, None, None, None]
    t.set_populations(A)
    p0 = t.totals()
    t.step(1)
    f = t.ib_force()
    area = t.vertex_weights().sum()
    np.testing.assert_allclose(f.reshape(3, -1).sum(axis=1), -U * area, rtol=1e-12, atol=0)
    p1 = t.totals()
    np.testing.assert_allclose(p1[1:] - p0[1:], f.reshape(3, -1).sum(axis=1), rtol=1e-10, atol=1e-20)
    assert abs(p1[0] - p0[0]) < 1e-13


def test_spread_force_is_local_and_follows_the_delta():
    """Vertices at known points (a tiny triangle) spread into their 4 x 4 x 4
    nodes only, with weights phi(dx) phi(dy) phi(dz), phi(r) = (1 + cos(pi
    r/2))/4, written out here node by node."""
    U = np.array([1e-4, 0.0, 0.0])
    t = tube3d.Tube(12, 12, 12, 1.0, 0.0, geom=tube3d.BOX)
    # a degenerate 'body': one vertex with a triangle of area 3 around it
    xyz = np.array([[5.3, 6.6, 4.2], [5.3 + 1e-9, 6.6, 4.2], [5.3, 6.6 + 1e-9, 4.2]])
    tri = np.array([[0, 1, 2]])
    t.add_fixed_body(xyz, tri)
    A = t.populations()
    A[:] = tube3d.heq(0.0, *U)[:, None, None, None]
    t.set_populations(A)
    t.step(1)
    f = t.ib_force()[0]
    w = t.vertex_weights()
    phi = lambda r: np.where(np.abs(r) < 2, 0.25 * (1 + np.cos(np.pi * np.abs(r) / 2)), 0.0)
    want = np.zeros_like(f)
    for v in range(3):
        for z in range(12):
            for y in range(12):
                for x in range(12):
                    W = phi(xyz[v, 0] - x) * phi(xyz[v, 1] - y) * phi(xyz[v, 2] - z)
                    want[z, y, x] += W * (-U[0]) * w[v]
    np.testing.assert_allclose(f, want, rtol=1e-9, atol=1e-22)
    assert np.count_nonzero(np.abs(f) > 0) <= 5 * 5 * 5
