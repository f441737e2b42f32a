"""Pins of the oracle's immersed-boundary, membrane, integrator and bond parts
(no GPU).  Each test names the passage it checks and the property that fixes
the result independently of the oracle's own code."""
import json
import os

import numpy as np
import pytest

import oracle
from helpers import oracle_sim
from paper_2210_06043_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
KAT = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")))


# ---- cosine delta kernel --------------------------------------------------------------

def test_phi_values():
    """phi(r) = (1 + cos(pi r/2))/4 on |r| <= 2: phi(0) = 1/2, phi(1) = 1/4,
    phi(2) = 0, symmetric, zero outside."""
    assert oracle.phi(0.0) == 0.5
    assert abs(oracle.phi(1.0) - 0.25) < 1e-16 and abs(oracle.phi(-1.0) - 0.25) < 1e-16
    assert oracle.phi(2.0) == 0.0 and oracle.phi(-2.5) == 0.0 and oracle.phi(3.0) == 0.0
    for r in np.linspace(-2, 2, 41):
        assert abs(oracle.phi(r) - oracle.phi(-r)) < 1e-16


@pytest.mark.parametrize("s", [0.0, 0.13, 0.25, 0.5, 0.77, 0.999])
def test_phi_moment_identities(s):
    """Over the four nodes of a stencil, sum phi = 1 and sum phi^2 = 3/8 for
    every shift s, and the first moment is s - 1/2 + (cos(pi s/2) - sin(pi s/2))/2
    (not zero: the kernel does not reproduce linear fields exactly)."""
    r = np.array([1 + s, s, s - 1, s - 2])
    p = np.array([oracle.phi(v) for v in r])
    assert abs(p.sum() - 1) < 1e-15
    assert abs((p ** 2).sum() - 0.375) < 1e-15
    m1 = s - 0.5 + 0.5 * (np.cos(np.pi * s / 2) - np.sin(np.pi * s / 2))
    assert abs((p * r).sum() - m1) < 1e-15


def test_stencil_equals_brute_force():
    """Periodic 9x8 grid: the 16 stencil weights equal phi(X-i) phi(Y-j)
    evaluated at every node of the grid (nodes outside the stencil have zero
    weight), for points anywhere including across the periodic seam."""
    nx, ny = 9, 8
    s = oracle.Sim(nx, ny, 1.0, 0, 0, walls=0)
    rng = np.random.default_rng(7)
    for X, Y in list(rng.uniform(-3, 12, (20, 2))) + [(0.0, 0.0), (8.999, 7.5)]:
        ii, jj, w = s.stencil(X, Y)
        dense = np.zeros((ny, nx))
        for b in range(4):
            for a in range(4):
                dense[jj[b], ii[a]] += w[b, a]
        brute = np.zeros((ny, nx))
        for j in range(-ny, 2 * ny):
            for i in range(-nx, 2 * nx):
                brute[j % ny, i % nx] += oracle.phi(X - i) * oracle.phi(Y - j)
        np.testing.assert_allclose(dense, brute, atol=1e-15)


def test_stencil_wall_rows():
    """Stencils that cross a wall (the paper is silent): points are clamped to
    Y in [-1, ny].  For the probes the rows beyond the wall are dropped and
    the fluid rows renormalised to sum 1.  For the velocity coupling a row
    beyond the wall is the odd image of the fluid row mirrored about the
    wall (below y = -1/2: row -1-j; above y = ny - 1/2: row 2 ny - 1 - j)
    with its full kernel weight negated, so the weights sum to the fluid
    share minus the image share."""
    ny = 6
    s = oracle.Sim(10, ny, 1.0, 0, 0, walls=3)
    for Y in [-1.5, -1.0, -0.4, 0.3, 2.5, 4.6, 5.2, 6.0, 7.0]:
        Yc = min(max(Y, -1.0), float(ny))
        j0 = int(np.floor(Yc)) - 1
        rows = [j0 + b for b in range(4)]
        full = np.array([oracle.phi(Yc - j) for j in rows])
        fluid = np.array([full[b] if 0 <= rows[b] < ny else 0.0 for b in range(4)])
        px = np.array([oracle.phi(4.3 - (3 + a)) for a in range(4)])
        ii, jj, w = s.stencil(4.3, Y, oracle.STEN_PROBE)
        assert abs(w.sum() - 1) < 1e-15
        np.testing.assert_allclose(w, np.outer(fluid, px) / (fluid.sum() * px.sum()), atol=1e-15)
        ii, jj, w = s.stencil(4.3, Y, oracle.STEN_VELOCITY)
        sign = np.array([1.0 if 0 <= j < ny else -1.0 for j in rows])
        mirror = [j if 0 <= j < ny else (-1 - j if j < 0 else 2 * ny - 1 - j) for j in rows]
        np.testing.assert_allclose(w, np.outer(sign * full, px) / (full.sum() * px.sum()), atol=1e-15)
        assert list(jj) == mirror
        if 1.0 <= Yc <= ny - 2.0:             # away from the walls all readings agree
            assert abs(w.sum() - 1) < 1e-15


def test_velocity_image_vanishes_on_the_walls():
    """With the odd image the interpolated velocity is zero on the walls
    themselves (y = -1/2 and y = ny - 1/2) for any fluid field: no slip."""
    ny = 9
    s = oracle.Sim(12, ny, 1.0, 0, 0, walls=3)
    rng = np.random.default_rng(4)
    f = rng.standard_normal((ny, 12))
    for X in (0.3, 5.0, 7.77):
        assert abs(s.interp_field(f, X, -0.5)) < 1e-15
        assert abs(s.interp_field(f, X, ny - 0.5)) < 1e-15


def test_velocity_image_reproduces_wall_shear():
    """A shear flow u = c (y + 1/2), zero on the lower wall, is its own odd
    image: near the wall the interpolation equals the unbounded kernel's,
    c (Y + 1/2 - m1(frac Y)), so the near-wall stencil loses nothing of a
    linear profile (the wall-nodes-at-rest reading would)."""
    ny, c = 10, 0.37
    s = oracle.Sim(8, ny, 1.0, 0, 0, walls=3)
    f = c * (np.arange(ny)[:, None] + 0.5) * np.ones((ny, 8))
    m1 = lambda t: t - 0.5 + 0.5 * (np.cos(np.pi * t / 2) - np.sin(np.pi * t / 2))
    for Y in (-0.45, -0.1, 0.0, 0.3, 0.9, 1.6):
        expect = c * (Y + 0.5 - m1(Y - np.floor(Y)))
        assert abs(s.interp_field(f, 3.2, Y) - expect) < 1e-14


def test_interp_linear_field_closed_form():
    """Interpolating f = a + b x + c y (periodic box, point away from the
    seam) gives a + b (X - m1(sx)) + c (Y - m1(sy)) with the kernel's first
    moment m1(s) = s - 1/2 + (cos(pi s/2) - sin(pi s/2))/2: pins the node
    indexing and the x/y roles of the weights."""
    nx, ny = 16, 14
    s = oracle.Sim(nx, ny, 1.0, 0, 0, walls=0)
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    a, b, c = 0.3, -0.7, 1.9
    f = a + b * xx + c * yy
    m1 = lambda t: t - 0.5 + 0.5 * (np.cos(np.pi * t / 2) - np.sin(np.pi * t / 2))
    for X, Y in [(5.25, 6.6), (7.0, 3.1), (8.9, 9.45)]:
        sx, sy = X - np.floor(X), Y - np.floor(Y)
        expect = a + b * (X - m1(sx)) + c * (Y - m1(sy))
        assert abs(s.interp_field(f, X, Y) - expect) < 1e-12


def test_spread_is_adjoint_of_interp():
    """Spreading uses the weights of interpolation at x^n: for any node field
    u, sum_x f_ib(x) u(x) = sum_v dV_v F_v . u(X_v) (checked on the spread
    force of one coupled step with an arbitrary u)."""
    cfg = inputs.config_tiny()
    s = oracle_sim(cfg)
    s.step(3)
    xs = [s.vertices(k).copy() for k in range(len(cfg.bodies))]
    s.step(1)
    f = s.node_fields()
    rng = np.random.default_rng(3)
    u = rng.standard_normal((cfg.ny, cfg.nx))
    v = rng.standard_normal((cfg.ny, cfg.nx))
    lhs = (f["fibx"] * u).sum() + (f["fiby"] * v).sum()
    rhs = 0.0
    for k in range(len(cfg.bodies)):
        w = s.body_work(k)
        x = xs[k]
        seg = np.hypot(*(np.roll(x, -1, 0) - x).T)
        dV = 0.5 * (seg + np.roll(seg, 1))
        F = dV[:, None] * (w["U"] - w["ustar"])
        for q in range(len(x)):
            rhs += F[q, 0] * s.interp_field(u, *x[q]) + F[q, 1] * s.interp_field(v, *x[q])
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1e-30) + 1e-20


# ---- membrane mechanics ---------------------------------------------------------------

def _wobbly(n=48, R=6.0, seed=0, amp=0.15):
    rest = inputs.circle(n, R, 10.0, 9.0)
    rng = np.random.default_rng(seed)
    return rest + amp * rng.standard_normal(rest.shape), rest


def test_membrane_forces_vanish_at_rest():
    """Eqs. (8), (10), (11) vanish in the stress-free configuration
    (l = l0, theta = theta0, A = A0)."""
    for xy in [inputs.circle(40, 5.0, 3.0, 4.0), inputs.biconcave(64, 20.0, 0, 0),
               inputs.rectangle(48, 10.0, 4.0, 0.0, 0.0)]:
        f = oracle.membrane_forces(xy, xy, ks=0.3, kb=0.05, ka=1.0, pref=1 / 3)
        assert np.abs(f).max() < 1e-14


def test_membrane_forces_sum_and_torque():
    """Spring pairs are equal and opposite, bending weights sum to
    l/(l+r) + r/(l+r) - 1 = 0, and sum_l n_l l_l = 0 on a closed polygon, so
    the internal forces of a body sum to zero; springs and the area penalty
    (a uniform pressure) also exert no net torque."""
    xy, rest = _wobbly()
    f = oracle.membrane_forces(xy, rest, ks=0.3, kb=0.05, ka=1.0, pref=1 / 3)
    assert np.abs(f.sum(0)).max() < 1e-14
    f2 = oracle.membrane_forces(xy, rest, ks=0.3, kb=0.0, ka=1.0, pref=1 / 3)
    torque = np.sum(xy[:, 0] * f2[:, 1] - xy[:, 1] * f2[:, 0])
    assert abs(torque) < 1e-13
    fb = oracle.membrane_forces(xy, rest, ks=0.0, kb=0.05, ka=0.0, pref=1 / 3)
    assert np.abs(fb).max() > 1e-4            # bending is active on the wobbly shape
    assert np.abs(fb.sum(0)).max() < 1e-15


@pytest.mark.parametrize("shift", [0.0, 24.0])
def test_repulsion_closed_form(shift):
    """Eq. (12) by brute force over the vertex pairs of two rigid circles at
    rest: switching the prefactor on changes the force on vertex v by
    -sum_u pref d_uv^(-5/2) n_v over the partners u closer than the cut-off,
    with n_v the radial unit vector of a regular polygon.  shift = 24 puts
    the contact on the periodic seam (one body stored wrapped)."""
    cfg = inputs.config_contact(kinds=(inputs.RIGID, inputs.RIGID))
    for b in cfg.bodies:
        b.xy = b.xy + np.array([shift, 0.0])
        if b.xy[:, 0].min() >= cfg.nx:
            b.xy = b.xy - np.array([cfg.nx, 0.0])
    pref = cfg.rep_pref
    forces = []
    for p in (pref, 0.0):
        cfg.rep_pref = p
        s = oracle_sim(cfg)
        s.step(1)
        forces.append([s.body_work(k)["force"] for k in (0, 1)])
    xy = [b.xy for b in cfg.bodies]
    centre = [x.mean(0) for x in xy]
    hits = 0
    for k in (0, 1):
        other = xy[1 - k]
        nrm = (xy[k] - centre[k]) / np.linalg.norm(xy[k] - centre[k], axis=1)[:, None]
        expect = np.zeros_like(xy[k])
        for v in range(len(xy[k])):
            dx = xy[k][v, 0] - other[:, 0]
            dx -= cfg.nx * np.round(dx / cfg.nx)
            d = np.hypot(dx, xy[k][v, 1] - other[:, 1])
            close = d < cfg.rep_cut
            hits += close.sum()
            expect[v] = -np.sum(pref * d[close] ** -2.5) * nrm[v]
        np.testing.assert_allclose(forces[0][k] - forces[1][k], expect, rtol=0, atol=1e-15)
    assert hits == 6          # three pairs, seen from both sides


def test_spring_and_area_forces_are_gradients():
    """Eq. (8) is -dV/dx of V = sum k_s (l - l0)^2 / 2 (Eq. 7), and the area
    penalty of Eq. (11), split half to each vertex, is -dV/dx of
    V = k_a p_ref A0 (1 - A/A0)^2 / 2: central finite differences."""
    xy, rest = _wobbly(n=24, seed=2, amp=0.3)
    ks, ka, pref = 0.7, 1.3, 1 / 3
    A0 = abs(oracle.polygon(rest)["area"])
    l0 = np.hypot(*(np.roll(rest, -1, 0) - rest).T)

    def V(p):
        l = np.hypot(*(np.roll(p, -1, 0) - p).T)
        x, y = p[:, 0], p[:, 1]
        A = 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)
        return 0.5 * ks * np.sum((l - l0) ** 2) + 0.5 * ka * pref * A0 * (1 - A / A0) ** 2

    f = oracle.membrane_forces(xy, rest, ks=ks, kb=0.0, ka=ka, pref=pref)
    h = 1e-6
    num = np.zeros_like(xy)
    for v in range(len(xy)):
        for d in range(2):
            p, m = xy.copy(), xy.copy()
            p[v, d] += h
            m[v, d] -= h
            num[v, d] = -(V(p) - V(m)) / (2 * h)
    np.testing.assert_allclose(f, num, rtol=1e-6, atol=1e-8)


def test_bending_restores_and_points_along_vertex_normal():
    """Eq. (10): a single vertex pushed outward (theta > theta0) feels
    -k_b (theta - theta0) n_v (inward), its neighbours share the opposite
    amount in the ratios l/(l+r) and r/(l+r)."""
    rest = inputs.circle(32, 6.0, 0, 0)
    xy = rest.copy()
    xy[5] *= 1.05
    kb = 0.2
    f = oracle.membrane_forces(xy, rest, ks=0.0, kb=kb, ka=0.0, pref=0)
    g = oracle.polygon(xy)
    g0 = oracle.polygon(rest)
    dth = g["theta"][5] - g0["theta"][5]
    assert dth > 0
    nv = g["nv"][5]
    # vertex 5 receives its own term plus the neighbour terms of vertices 4 and 6
    own = -kb * dth * nv
    assert np.dot(f[5], nv) < 0
    l_, r_ = g["length"][4], g["length"][5]
    contrib4 = kb * dth * l_ / (l_ + r_) * nv
    contrib6 = kb * dth * r_ / (l_ + r_) * nv
    # neighbours 4 and 6 also have their own angle changes; check the sum instead
    assert np.abs(f.sum(0)).max() < 1e-15
    assert np.dot(own + contrib4 + contrib6, nv) == pytest.approx(0.0, abs=1e-15)


def test_bending_share_follows_eq10_not_its_mirror():
    """Eq. (10) gives the left neighbour the share l_left/(l_left + l_right).
    The mirrored assignment (left gets l_right/(...)) would make every
    three-vertex bending stencil torque-free, since its weighted sum of
    neighbour offsets is parallel to n_v; the paper's assignment is torque-free
    only when l_left = l_right.  A polygon with unequal edges and bending only
    must therefore show a net torque, and the same polygon with equal edges
    (a regular polygon scaled radially at one vertex pair symmetric) none."""
    rest = inputs.circle(12, 4.0, 0.0, 0.0)
    xy = rest.copy()
    xy[3] = xy[3] + 0.6 * (xy[4] - xy[3])          # vertex 3 slides along its edge: unequal lengths
    f = oracle.membrane_forces(xy, rest, ks=0.0, kb=0.1, ka=0.0, pref=0)
    torque = np.sum(xy[:, 0] * f[:, 1] - xy[:, 1] * f[:, 0])
    assert abs(torque) > 1e-6
    sym = rest * np.where(np.arange(12)[:, None] % 2 == 0, 1.1, 1.0)  # alternating radii, equal edges
    fs = oracle.membrane_forces(sym, rest, ks=0.0, kb=0.1, ka=0.0, pref=0)
    assert abs(np.sum(sym[:, 0] * fs[:, 1] - sym[:, 1] * fs[:, 0])) < 1e-15


def test_shapes_closed_forms():
    """Regular n-gon area (n/2) R^2 sin(2 pi/n) and perimeter 2 n R sin(pi/n);
    the biconcave section of Eq. (21) (a alpha = 1): perimeter 4.9288,
    area 0.89123, reduced area 4 pi A/P^2 = 0.46101 (the paper states 0.481;
    its printed formula gives 0.461)."""
    n, R = 37, 3.3
    g = oracle.polygon(inputs.circle(n, R, 1.0, 2.0))
    assert abs(g["area"] - n / 2 * R ** 2 * np.sin(2 * np.pi / n)) < 1e-12
    assert abs(g["perimeter"] - 2 * n * R * np.sin(np.pi / n)) < 1e-12
    assert abs(g["cx"] - 1.0) < 1e-12 and abs(g["cy"] - 2.0) < 1e-12
    b = oracle.polygon(inputs.biconcave(8192, 1.0, 0.0, 0.0))
    assert b["area"] > 0                       # counter-clockwise after reversal
    assert abs(b["perimeter"] - 4.9288) < 1e-4
    assert abs(b["area"] - 0.89123) < 1e-5
    assert abs(4 * np.pi * b["area"] / b["perimeter"] ** 2 - 0.46101) < 1e-5
    co = GOLD["biconcave_coefficients"]["value"]
    assert co == [0.207, 2.003, 1.123]


def test_polar_moment_closed_form():
    """Rectangle b x h about its centroid: J = b h (b^2 + h^2)/12."""
    b, h = 6.0, 2.0
    xy = inputs.rectangle(64, b, h, 1.0, 0.0)
    g = oracle.polygon(xy)
    assert abs(oracle.polar_moment(xy, g["cx"], g["cy"]) - b * h * (b * b + h * h) / 12) < 1e-11


# ---- integrators (Eqs. 17-20) ---------------------------------------------------------

def _one_body_sim(kind, xy, rho_r=1.0):
    s = oracle.Sim(16, 16, 1.0, 0, 0, walls=0)
    s.add_body(kind, xy, None, rho_r=rho_r)
    return s


def test_deformable_free_drift():
    """Eq. (17) with F = 0 and a uniform interpolated velocity u*: the
    vertices move by u* per step; Eq. (18) gives U = 1.5 u* on the first step
    (released at rest) and U = u* afterwards."""
    xy = inputs.circle(12, 3.0, 8.0, 8.0)
    s = _one_body_sim(inputs.DEFORMABLE, xy)
    u = np.array([1.3e-3, -0.4e-3])
    for n in range(1, 6):
        s.set_body_work(0, ustar=np.tile(u, (12, 1)), force=np.zeros((12, 2)))
        s.integrate_body(0)
        np.testing.assert_allclose(s.vertices(0), xy + n * u, rtol=0, atol=1e-14)
        U = s.body_work(0)["U"]
        np.testing.assert_allclose(U, np.tile(1.5 * u if n == 1 else u, (12, 1)), rtol=1e-12)


def test_deformable_constant_force():
    """Eq. (17) with u* = 0 and constant F: each step moves F/(2 m_v),
    m_v = rho_r A0 / n (membrane mass spread over the vertices, Sec. 2.7)."""
    xy = inputs.circle(10, 2.0, 8.0, 8.0)
    s = _one_body_sim(inputs.DEFORMABLE, xy, rho_r=1.1)
    F = np.array([2e-4, 5e-5])
    mv = 1.1 * oracle.polygon(xy)["area"] / 10
    assert abs(s.body_diag(0)["vmass"] - mv) < 1e-14
    for n in range(1, 4):
        s.set_body_work(0, ustar=np.zeros((10, 2)), force=np.tile(F, (10, 1)))
        s.integrate_body(0)
        np.testing.assert_allclose(s.vertices(0), xy + n * 0.5 * F / mv, atol=1e-14)


def test_rigid_constant_force_bdf2_closed_form():
    """Eqs. (19)-(20) with a constant force from rest: u_n = (2/3)(2 u_{n-1}
    - u_{n-2}/2 + a) with a = F/m has the closed form
    u_n = a (n - 1/2 + 3^-n / 2); the centroid moves by u_n each step
    (x_c += u dt) and the vertices follow rigidly."""
    xy = inputs.ellipse(20, 3.0, 1.0, 8.0, 8.0)
    s = _one_body_sim(inputs.RIGID, xy, rho_r=1.1)
    g = oracle.polygon(xy)
    m = 1.1 * g["area"]
    F = np.array([3e-4, -1e-4])
    a = F / m
    pos = np.array([g["cx"], g["cy"]])
    for n in range(1, 8):
        s.set_body_work(0, force=np.tile(F / 20, (20, 1)))
        s.integrate_body(0)
        un = a * (n - 0.5 + 0.5 * 3.0 ** (-n))
        r = s.rigid(0)
        np.testing.assert_allclose([r["ucx"], r["ucy"]], un, rtol=1e-12)
        pos = pos + un
        np.testing.assert_allclose([r["xc"], r["yc"]], pos, rtol=1e-13)
        assert abs(r["phi"]) < 1e-15             # uniform force about the centroid: no torque
        np.testing.assert_allclose(s.vertices(0), xy + (pos - [g["cx"], g["cy"]]), atol=1e-13)
        np.testing.assert_allclose(s.body_work(0)["U"], np.tile(un, (20, 1)), rtol=1e-12)


def test_rigid_torque_bdf2_closed_form():
    """Eq. (20) with a constant moment M = sum (x - x_c) x F from a couple:
    omega_n = (M/I)(n - 1/2 + 3^-n/2), I = rho_r J0 (polar moment);
    phi accumulates omega, and U = u + omega z x (x - x_c)."""
    xy = inputs.ellipse(24, 3.0, 1.5, 8.0, 8.0)
    s = _one_body_sim(inputs.RIGID, xy)
    g = oracle.polygon(xy)
    I = oracle.polar_moment(xy, g["cx"], g["cy"])
    F = np.zeros((24, 2))
    F[0] = [1e-4, 0.0]
    F[12] = [-1e-4, 0.0]
    M = np.sum((xy[:, 0] - g["cx"]) * F[:, 1] - (xy[:, 1] - g["cy"]) * F[:, 0])
    phi = 0.0
    for n in range(1, 6):
        s.set_body_work(0, force=F)
        s.integrate_body(0)
        om = M / I * (n - 0.5 + 0.5 * 3.0 ** (-n))
        r = s.rigid(0)
        assert r["om"] == pytest.approx(om, rel=1e-12)
        phi += om
        assert r["phi"] == pytest.approx(phi, rel=1e-12)
        c, sn = np.cos(phi), np.sin(phi)
        rel = xy - [g["cx"], g["cy"]]
        exp = np.stack([c * rel[:, 0] - sn * rel[:, 1], sn * rel[:, 0] + c * rel[:, 1]], 1) + [r["xc"], r["yc"]]
        np.testing.assert_allclose(s.vertices(0), exp, atol=1e-13)
        d = s.vertices(0) - [r["xc"], r["yc"]]
        np.testing.assert_allclose(s.body_work(0)["U"], np.stack([-om * d[:, 1], om * d[:, 0]], 1) +
                                   [r["ucx"], r["ucy"]], atol=1e-18)


def test_area_penalty_relaxation():
    """Sec. 2.3: with k_a = 1 a body inflated away from A0 and left alone
    (fluid frozen, internal forces only) returns towards A0 monotonically."""
    rest = inputs.circle(64, 8.0, 20.0, 20.0)
    start = 20.0 + (rest - 20.0) * 1.03
    _, hist = oracle.relax_membrane(start, rest, ks=0.0, kb=0.0, ka=1.0, pref=1 / 3, rho_r=1.0, nsteps=400)
    A0 = oracle.polygon(rest)["area"]
    dev = np.abs(hist / A0 - 1)
    assert dev[0] > 0.05
    assert np.all(np.diff(dev) <= 1e-15)
    assert dev[-1] < 0.1 * dev[0]


# ---- bonds and the counter-based generator ---------------------------------------------

def test_philox_known_answers():
    """Philox4x32-10 against the published known-answer vectors."""
    for v in KAT["vectors"]:
        out = oracle.philox4x32_10([int(x, 16) for x in v["ctr"]], [int(x, 16) for x in v["key"]])
        assert out == [int(x, 16) for x in v["out"]]


def test_uniform_stream_properties():
    """The per-site draws are uniform on [0, 1) with 24-bit resolution."""
    r = np.array([oracle.uniform(42, n, s) for n in range(50) for s in range(200)])
    assert r.min() >= 0 and r.max() < 1
    assert np.all(np.round(r * 2 ** 24) == r * 2 ** 24)
    assert abs(r.mean() - 0.5) < 4 * np.sqrt(1 / 12 / len(r))
    assert abs(r.var() - 1 / 12) < 0.01


def _bonded_fixed_plate(ns=200, kr0=0.0, kf=0.0, seed=5, lift=0.0):
    s = oracle.Sim(40, 12, 1.0, 0.0, 0.0, walls=3)
    xy = inputs.rectangle(40, 30.0, 3.0, 20.0, -0.5 + 0.1 + lift)
    s.add_body(inputs.FIXED, xy)
    host, frac = inputs.place_sites(xy, ns if lift == 0.0 else ns, 0.3) if lift == 0.0 else (None, None)
    return s, xy, host, frac


def test_bonds_frozen_without_rates():
    """Sec. 2.5: with k_f = k_r0 = 0 no bond forms or breaks."""
    s = oracle.Sim(40, 12, 1.0, 1e-7, 0.0, walls=3)
    xy = inputs.rectangle(40, 30.0, 3.0, 20.0, -0.4)
    s.add_body(inputs.FIXED, xy)
    host, frac = inputs.place_sites(xy, 60, 0.3)
    s.add_bonds(0, host, frac, 1e-3, 0.3, 0.15, 0.0, 0.0, 0.01, 9)
    st0, an0 = s.bonds(0)
    assert st0.sum() == 60
    s.step(30)
    st1, an1 = s.bonds(0)
    assert np.array_equal(st0, st1) and np.array_equal(an0, an1)


def test_bond_survival_binomial():
    """Constant stretch, no re-binding (k_f = 0): every bound site breaks with
    the same probability P_r = 1 - exp(-k_r0 exp(|y_l - y_eq|/l_B)) per step,
    so after n steps the count is Binomial(N0, (1 - P_r)^n)."""
    s = oracle.Sim(40, 12, 1.0, 0.0, 0.0, walls=3)
    xy = inputs.rectangle(40, 30.0, 3.0, 20.0, -0.3)
    s.add_body(inputs.FIXED, xy)
    host, frac = inputs.place_sites(xy, 120, 0.4)
    ycr, yeq, lb, kr0 = 0.4, 0.1, 0.05, 0.004
    s.add_bonds(0, host, frac, 0.0, ycr, yeq, 0.0, kr0, lb, 11)
    st, _ = s.bonds(0)
    assert st.sum() == 120
    # every bound site on the flat base has gap 0.2, i.e. stretch 0.1
    Pr = 1 - np.exp(-kr0 * np.exp(0.1 / lb))
    n = 40
    s.step(n)
    k = s.count_bound(0)
    p = (1 - Pr) ** n
    # the two base corners carry sites on the short sides with a larger gap;
    # allow for them within a 5-sigma band
    mean, sd = 120 * p, np.sqrt(120 * p * (1 - p))
    assert abs(k - mean) < 5 * sd + 4


def test_c1_sites_and_constants():
    """The small workload's parameters follow Sec. 2.5 and 3.1: y_cr = 25 nm
    over dx = 0.125 um, y_eq = y_cr/2, sigma = nu^2/H, k_f/k_r0 = 8.5e3,
    rho_P/rho = 1.1, Ca = 1e-3, 50 sites engaged at t = 0."""
    cfg = inputs.config_c1()
    bd = cfg.bonds[0]
    assert bd.ycr == pytest.approx(GOLD["y_cr_m"]["value"] / 0.125e-6)
    assert bd.yeq == pytest.approx(GOLD["y_eq_over_y_cr"]["value"] * bd.ycr)
    assert bd.kf / bd.kr0 == pytest.approx(GOLD["kf_over_kr0"]["value"])
    assert bd.sigma == pytest.approx((1 / 6) ** 2 / 60)
    assert cfg.bodies[1].rho_r == GOLD["particle_density_ratio"]["value"]
    nu, umax = cfg.meta["nu"], cfg.meta["umax"]
    assert umax * 60 / nu == pytest.approx(GOLD["reynolds"]["value"])
    assert nu * umax / cfg.bodies[0].ks == pytest.approx(GOLD["capillary_number"]["value"])
    assert cfg.rep_pref == pytest.approx(GOLD["repulsion_prefactor"]["value"])
    assert cfg.probe_dist == GOLD["probe_length"]["value"]
    s = oracle_sim(cfg)
    assert s.count_bound(1) == 50
    # physical Reynolds number of Sec. 3.1
    Re = GOLD["centreline_speed_ms"]["value"] * GOLD["channel_height_m"]["value"] / \
        GOLD["kinematic_viscosity_m2s"]["value"]
    assert Re == pytest.approx(GOLD["reynolds"]["value"])


def test_coupled_step_invariants():
    """Full coupled steps of the small channel (parity unpinned beyond the
    invariants): mass constant, no vertex leaves the fluid, N_L stays within
    the site count, the deformable cell keeps its area to k_a = 1 accuracy."""
    cfg = inputs.config_tiny()
    s = oracle_sim(cfg)
    m0 = s.totals()[0]
    A0 = s.body_diag(0)["A0"]
    s.step(200)
    assert abs(s.totals()[0] - m0) < 1e-15 * 9 * cfg.nx * cfg.ny
    assert s.flags == 0
    assert 0 <= s.count_bound(1) <= len(cfg.bonds[0].host)
    assert abs(s.body_diag(0)["area"] / A0 - 1) < 1e-2
