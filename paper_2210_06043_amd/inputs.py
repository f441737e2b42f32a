"""Seeded synthetic inputs shaped like the paper's capillary workloads.

This module is the only code shared by the HIP path and the FP64 oracle, and
it holds none of the method's arithmetic: it maps the physical set-up of
Sec. 3.1 to lattice parameters, draws membrane shapes and ligand sites, and
returns plain arrays.  Both sides receive identical numbers from here and
compute everything else themselves.

Lattice units throughout: dx = dt = 1, rho_0 = 1, c_s^2 = 1/3.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

DEFORMABLE, RIGID, FIXED = 0, 1, 2
TAG_CELL, TAG_PARTICLE = 1, 2

# Eq. (12) prefactor; minimum allowed vertex distance dx; probe length 1.2 dx (Sec. 2.6)
REP_PREFACTOR = 1.0e-4 / (8.0 * np.sqrt(2.0))
REP_CUTOFF = 1.0
PROBE_DIST = 1.2
P_REF = 1.0 / 3.0          # reference pressure c_s^2 rho_0 of the area penalty
KA = 1.0                   # incompressibility coefficient k_a (Sec. 2.3)
Y_CR_M = 25e-9             # critical bond gap, 25 nm (Sec. 2.5)
KF_OVER_KR0 = 8.5e3        # biochemical affinity k_f / k_r0 (Sec. 3.1)


@dataclass
class Body:
    kind: int
    xy: np.ndarray                    # (n, 2) counter-clockwise, unwrapped lattice coordinates
    xy_rest: Optional[np.ndarray]     # stress-free shape or None (= xy)
    ks: float = 0.0
    kb: float = 0.0
    ka: float = KA
    pref: float = P_REF
    rho_r: float = 1.0
    tag: int = 0


@dataclass
class Bonds:
    body: int
    host: np.ndarray                  # (ns,) int32 element index (element e joins vertex e to e+1)
    frac: np.ndarray                  # (ns,) position along the element, [0, 1)
    sigma: float
    ycr: float
    yeq: float
    kf: float
    kr0: float
    lb: float
    seed: int


@dataclass
class Config:
    name: str
    nx: int
    ny: int
    tau: float
    gx: float
    gy: float = 0.0
    walls: int = 3
    ux_init: Optional[np.ndarray] = None   # (ny,) initial x-velocity per row, None = rest
    bodies: List[Body] = field(default_factory=list)
    bonds: List[Bonds] = field(default_factory=list)
    rep_pref: float = REP_PREFACTOR
    rep_cut: float = REP_CUTOFF
    probe_dist: float = PROBE_DIST
    steps: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_vertices(self):
        return sum(len(b.xy) for b in self.bodies)

    @property
    def n_sites(self):
        return sum(len(b.host) for b in self.bonds)


# ---- parameter mapping (Sec. 3.1) -------------------------------------------------

def viscosity(tau):
    """nu = c_s^2 (tau - 1/2) dt (Sec. 2.1)."""
    return (tau - 0.5) / 3.0


def channel(H, Re, tau):
    """Centre-line speed and driving body force of a channel of height H
    (lattice nodes) at Reynolds number Re = u_max H / nu (Sec. 3.1):
    u_max = Re nu / H and g = 8 nu u_max / H^2 (plane Poiseuille flow)."""
    nu = viscosity(tau)
    umax = Re * nu / H
    g = 8.0 * nu * umax / H ** 2
    return nu, umax, g


def poiseuille_profile(ny, g, tau):
    """Steady x-velocity per row of the body-force driven channel with
    halfway bounce-back walls at y = -1/2 and y = ny - 1/2: the parabola plus
    the lattice slip of BGK bounce-back, g (16 Lambda - 3) / (24 nu) with
    Lambda = (tau - 1/2)^2 (used only as an initial condition)."""
    nu = viscosity(tau)
    H = float(ny)
    eta = np.arange(ny) + 0.5
    lam = (tau - 0.5) ** 2
    return g / (2 * nu) * eta * (H - eta) + g * (16 * lam - 3) / (24 * nu)


def stiffness(umax, tau, Ca):
    """k_s from Ca = rho nu u_max / k_s (Sec. 3.1)."""
    return viscosity(tau) * umax / Ca


def bond_spring(tau, H, sigma_star=1.0):
    """sigma in lattice units from its dimensionless group rho nu^2 / H (Sec. 2.5)."""
    return sigma_star * viscosity(tau) ** 2 / H


# ---- shapes ----------------------------------------------------------------------------

def _resample(fx, fy, q0, q1, n, dense=200000):
    """n points on the closed curve (fx(q), fy(q)), q in [q0, q1), equally spaced in arc length."""
    q = np.linspace(q0, q1, dense + 1)
    x, y = fx(q), fy(q)
    s = np.concatenate([[0.0], np.cumsum(np.hypot(np.diff(x), np.diff(y)))])
    target = np.arange(n) * s[-1] / n
    qs = np.interp(target, s, q)
    return np.stack([fx(qs), fy(qs)], 1)


def circle(n, R, cx, cy, start=-np.pi / 2):
    t = start + 2 * np.pi * np.arange(n) / n
    return np.stack([cx + R * np.cos(t), cy + R * np.sin(t)], 1)


def ellipse(n, a, b, cx, cy):
    """Ellipse with semi-axes a (x) and b (y), counter-clockwise from the bottom, uniform in arc length."""
    return _resample(lambda q: cx + a * np.cos(q), lambda q: cy + b * np.sin(q),
                     -np.pi / 2, 1.5 * np.pi, n)


def biconcave(n, a_alpha, cx, cy, dense=200000):
    """Median section of a red blood cell, Eq. (21), with a*alpha the cell
    radius; reversed to counter-clockwise order; uniform in arc length."""
    fx = lambda q: cx - a_alpha * np.sin(q)        # x -> -x reverses the orientation
    fy = lambda q: cy + 0.5 * a_alpha * (0.207 + 2.003 * np.sin(q) ** 2 - 1.123 * np.sin(q) ** 4) * np.cos(q)
    return _resample(fx, fy, -0.5 * np.pi, 1.5 * np.pi, n, dense)


def rectangle(n, b, h, cx, y_bottom):
    """Discoidal particle section: a b x h rectangle, corners included, each
    side divided evenly, counter-clockwise from the bottom-left corner."""
    nb = int(round(n * b / (2 * (b + h))))
    nh = n // 2 - nb
    if nb < 1 or nh < 1 or 2 * (nb + nh) != n:
        raise ValueError("vertex count does not fit the rectangle")
    x0, x1, y0, y1 = cx - b / 2, cx + b / 2, y_bottom, y_bottom + h
    pts = []
    for k in range(nb):
        pts.append((x0 + b * k / nb, y0))
    for k in range(nh):
        pts.append((x1, y0 + h * k / nh))
    for k in range(nb):
        pts.append((x1 - b * k / nb, y1))
    for k in range(nh):
        pts.append((x0, y1 - h * k / nh))
    return np.array(pts, dtype=np.float64)


# ---- ligand sites ------------------------------------------------------------------------

def place_sites(xy, n_bound, ycr, wall_y=-0.5, dense=400000):
    """Ligand sites evenly spaced in arc length along the whole perimeter, with
    the spacing chosen so that exactly ``n_bound`` sites lie closer than ``ycr``
    to the wall at t = 0 (they are placed at the centres of n_bound equal parts
    of the arc where the gap is below ycr).  Returns (host element, fraction)."""
    xy = np.asarray(xy, dtype=np.float64)
    n = len(xy)
    nxt = np.roll(xy, -1, axis=0)
    seg = np.hypot(*(nxt - xy).T)
    s0 = np.concatenate([[0.0], np.cumsum(seg)])
    P = s0[-1]

    def point(s):
        s = np.mod(s, P)
        e = np.minimum(np.searchsorted(s0, s, side="right") - 1, n - 1)
        f = (s - s0[e]) / seg[e]
        return e, f, xy[e] + f[:, None] * (nxt[e] - xy[e])

    dense = np.linspace(0.0, P, dense + 1)[:-1]
    _, _, pts = point(dense)
    close = pts[:, 1] - wall_y < ycr
    if not close.any() or close.all():
        raise ValueError("no contiguous binding arc")
    # rotate so that the binding arc is contiguous and starts at index 0
    k0 = int(np.argmax(close & ~np.roll(close, 1)))
    roll = np.roll(close, -k0)
    m = int(np.argmin(roll))            # first not-close index after the run
    if roll[m:].any():
        raise ValueError("binding arc is not contiguous")
    ds = P / len(dense)
    a = dense[k0]
    length = m * ds
    spacing = length / n_bound
    total = int(np.floor(P / spacing))
    s = a + spacing * (np.arange(total) + 0.5)
    e, f, p = point(s)
    nclose = int(np.sum(p[:, 1] - wall_y < ycr))
    if nclose != n_bound:
        raise ValueError(f"site placement gave {nclose} bound sites, wanted {n_bound}")
    order = np.lexsort((f, e))
    return e[order].astype(np.int32), f[order]


# ---- workloads --------------------------------------------------------------------------------

def config_c1(seed=0, steps=2000):
    """Plain method, small: 480x60 channel (dx = 0.125 um, H = 7.5 um), tau = 1,
    Re = 0.01, walls top and bottom, periodic in x; one circular deformable
    cell (R = 28, 256 vertices, Ca = 1e-3, beta = 0.1) upstream; one rigid
    16x4 elliptical particle (64 vertices, rho_P/rho = 1.1) on the lower wall
    with 50 bonds engaged."""
    nx, ny, tau = 480, 60, 1.0
    nu, umax, g = channel(ny, 0.01, tau)
    dx_um = 7.5 / ny
    ks = stiffness(umax, tau, 1e-3)
    cell = Body(DEFORMABLE, circle(256, 28.0, 40.0, 29.5), None, ks=ks, kb=0.1 * ks, rho_r=1.0, tag=TAG_CELL)
    ycr = Y_CR_M / (dx_um * 1e-6)
    yeq = 0.5 * ycr
    part_xy = ellipse(64, 8.0, 2.0, 100.0, -0.5 + yeq + 2.0)
    part = Body(RIGID, part_xy, None, rho_r=1.1, tag=TAG_PARTICLE)
    host, frac = place_sites(part_xy, 50, ycr)
    kf = 8.5e-3
    bonds = Bonds(1, host, frac, sigma=bond_spring(tau, ny), ycr=ycr, yeq=yeq, kf=kf,
                  kr0=kf / KF_OVER_KR0, lb=ycr / 20.0, seed=seed)
    return Config("c1_480x60", nx, ny, tau, g, ux_init=poiseuille_profile(ny, g, tau),
                  bodies=[cell, part], bonds=[bonds], steps=steps,
                  meta=dict(umax=umax, nu=nu, dx_um=dx_um, n_bound0=50))


def config_c2(seed=0, steps=50000, ar=None, ca=None, cell_shift=0.0):
    """Paper-scale: 3840x240 channel (dx = 0.03125 um), Re = 0.01, tau = 1;
    six cells alternating biconcave and globular (radius 3.5 um = 112 nodes,
    512 vertices each) on the centre line at x = 320 + 640 k (+ cell_shift);
    one discoidal particle 2 um long (64 nodes), aspect ratio from {0.25,
    0.5, 1.0} and Ca from {0, 1e-4, 1e-3} drawn with the seed, 128 vertices,
    200 bonds engaged, mid-gap between the first two cells on the lower
    wall."""
    nx, ny, tau = 3840, 240, 1.0
    nu, umax, g = channel(ny, 0.01, tau)
    dx_um = 7.5 / ny
    rng = np.random.default_rng(seed)
    ar = float(rng.choice([0.25, 0.5, 1.0])) if ar is None else ar
    ca = float(rng.choice([0.0, 1e-4, 1e-3])) if ca is None else ca
    ks_cell = stiffness(umax, tau, 1e-3)
    bodies = []
    for k in range(6):
        cx = 320.0 + 640.0 * k + cell_shift
        xy = biconcave(512, 112.0, cx, 119.5) if k % 2 == 0 else circle(512, 112.0, cx, 119.5)
        bodies.append(Body(DEFORMABLE, xy, None, ks=ks_cell, kb=0.1 * ks_cell, rho_r=1.0, tag=TAG_CELL))
    ycr = Y_CR_M / (dx_um * 1e-6)
    yeq = 0.5 * ycr
    b, h = 64.0, ar * 64.0
    part_xy = rectangle(128, b, h, 640.0, -0.5 + yeq)
    if ca == 0.0:
        part = Body(RIGID, part_xy, None, rho_r=1.1, tag=TAG_PARTICLE)
    else:
        ks = stiffness(umax, tau, ca)
        part = Body(DEFORMABLE, part_xy, None, ks=ks, kb=0.1 * ks, rho_r=1.1, tag=TAG_PARTICLE)
    bodies.append(part)
    host, frac = place_sites(part_xy, 200, ycr)
    kf = 8.5e-3
    bonds = Bonds(6, host, frac, sigma=bond_spring(tau, ny), ycr=ycr, yeq=yeq, kf=kf,
                  kr0=kf / KF_OVER_KR0, lb=ycr / 20.0, seed=seed)
    return Config("c2_3840x240", nx, ny, tau, g, ux_init=poiseuille_profile(ny, g, tau),
                  bodies=bodies, bonds=[bonds], steps=steps,
                  meta=dict(umax=umax, nu=nu, dx_um=dx_um, ar=ar, ca=ca, n_bound0=200,
                            cell_types=[1, 0, 1, 0, 1, 0]))


def config_c2_placed(seed, k):
    """Member k of stream seed of the paper-scale surrogate data: the
    paper-scale channel with its particle's aspect ratio and Ca drawn as in
    config_c2 and the row of cells shifted along the channel by U(-150, 150)
    nodes (the cells stay clear of the particle), so that the cell-particle
    distance varies between members: at tau = 1 a paper-scale run barely
    moves its cells, so placement supplies the range of r."""
    rng = np.random.default_rng([seed, k, 7])
    shift = float(rng.uniform(-150.0, 150.0))
    return config_c2(seed=int(rng.integers(0, 2**31 - 1)), cell_shift=shift)


def config_mr(seed=2, steps=2000):
    """Single-lattice roofline case: a 16384 x 1024 channel (16.8 M nodes,
    1.2 GB of FP32 populations per step, far beyond the 256 MB last-level
    cache) at the paper-scale resolution dx = 0.03125 um, Re = 0.01, tau = 1;
    24 cells of the paper-scale size (radius 3.5 um = 112 nodes, 512
    vertices, biconcave and circular alternating) in four rows of six; one
    discoidal particle (64 x AR*64 nodes, 128 vertices, 200 bonds) on the
    lower wall, drawn as in the paper-scale workload from the seed."""
    nx, ny, tau = 16384, 1024, 1.0
    nu, umax, g = channel(ny, 0.01, tau)
    dx_um = 7.5 / 240
    rng = np.random.default_rng(seed)
    ar = float(rng.choice([0.25, 0.5, 1.0]))
    ca = float(rng.choice([0.0, 1e-4, 1e-3]))
    ks_cell = stiffness(umax, tau, 1e-3)
    bodies = []
    for r in range(4):
        for c in range(6):
            cx, cy = (c + 0.5) * nx / 6, (r + 0.5) * ny / 4
            xy = biconcave(512, 112.0, cx, cy) if (r + c) % 2 == 0 else circle(512, 112.0, cx, cy)
            bodies.append(Body(DEFORMABLE, xy, None, ks=ks_cell, kb=0.1 * ks_cell, rho_r=1.0, tag=TAG_CELL))
    ycr = Y_CR_M / (dx_um * 1e-6)
    yeq = 0.5 * ycr
    part_xy = rectangle(128, 64.0, ar * 64.0, nx / 12, -0.5 + yeq)
    if ca == 0.0:
        part = Body(RIGID, part_xy, None, rho_r=1.1, tag=TAG_PARTICLE)
    else:
        ks = stiffness(umax, tau, ca)
        part = Body(DEFORMABLE, part_xy, None, ks=ks, kb=0.1 * ks, rho_r=1.1, tag=TAG_PARTICLE)
    bodies.append(part)
    host, frac = place_sites(part_xy, 200, ycr)
    kf = 8.5e-3
    bonds = Bonds(len(bodies) - 1, host, frac, sigma=bond_spring(tau, ny), ycr=ycr, yeq=yeq, kf=kf,
                  kr0=kf / KF_OVER_KR0, lb=ycr / 20.0, seed=seed)
    return Config("mr_16384x1024", nx, ny, tau, g, ux_init=poiseuille_profile(ny, g, tau), bodies=bodies,
                  bonds=[bonds], steps=steps, meta=dict(umax=umax, nu=nu, dx_um=dx_um, ar=ar, ca=ca, n_bound0=200))


def c3_member(seed, k, ar=None, ca=None):
    """Member k of the batched ensemble: a 64-row capillary (Re = 0.01,
    tau = 1) of length U{256..2048}; 1-4 cells, biconcave or globular with
    equal odds, 128-256 markers at half-node spacing, Ca = 1e-3, evenly
    spaced on the centre line; one discoidal particle 16 nodes long with
    aspect ratio U[0.25, 1] and 64 markers, mid-gap after the first cell on
    the lower wall, rigid (Ca = 0) with probability 1/4 and otherwise soft
    with Ca log-uniform in [1e-5, 1e-3], 20 bonds engaged.  Drawn from the
    stream seed * 2^20 + k.  ar and ca, if given, replace the particle's
    drawn aspect ratio and Ca (0 = rigid) and leave everything else of the
    member as drawn (a variant of the same capillary)."""
    sid = seed * (1 << 20) + k
    rng = np.random.default_rng(sid)
    ny, tau = 64, 1.0
    nu, umax, g = channel(ny, 0.01, tau)
    nx = int(rng.integers(256, 2049))
    dx_um = 7.5 / ny
    ks_cell = stiffness(umax, tau, 1e-3)
    ncell = int(rng.integers(1, 5))
    bodies = []
    xs = [(j + 0.5) * nx / ncell for j in range(ncell)]
    types = []
    for j in range(ncell):
        n = int(rng.integers(128, 257))
        R = 0.5 * n / (2.0 * np.pi)
        cy = 0.5 * (ny - 1) + float(rng.uniform(-1.0, 1.0))
        bic = rng.random() < 0.5
        types.append(1 if bic else 0)
        xy = biconcave(n, R, xs[j], cy, dense=20000) if bic else circle(n, R, xs[j], cy)
        bodies.append(Body(DEFORMABLE, xy, None, ks=ks_cell, kb=0.1 * ks_cell, rho_r=1.0, tag=TAG_CELL))
    ar_d = float(rng.uniform(0.25, 1.0))
    rigid = rng.random() < 0.25
    ca_d = 0.0 if rigid else float(10.0 ** rng.uniform(-5.0, -3.0))
    ar = ar_d if ar is None else float(ar)
    ca = ca_d if ca is None else float(ca)
    rigid = ca == 0.0
    ycr = Y_CR_M / (dx_um * 1e-6)
    yeq = 0.5 * ycr
    px = xs[0] + 0.5 * nx / ncell
    part_xy = rectangle(64, 16.0, ar * 16.0, px, -0.5 + yeq)
    if rigid:
        bodies.append(Body(RIGID, part_xy, None, rho_r=1.1, tag=TAG_PARTICLE))
    else:
        ks = stiffness(umax, tau, ca)
        bodies.append(Body(DEFORMABLE, part_xy, None, ks=ks, kb=0.1 * ks, rho_r=1.1, tag=TAG_PARTICLE))
    host, frac = place_sites(part_xy, 20, ycr, dense=40000)
    kf = 8.5e-3
    bonds = Bonds(len(bodies) - 1, host, frac, sigma=bond_spring(tau, ny), ycr=ycr, yeq=yeq, kf=kf,
                  kr0=kf / KF_OVER_KR0, lb=ycr / 20.0, seed=sid)
    return Config(f"c3_{k}_{nx}x{ny}", nx, ny, tau, g, ux_init=poiseuille_profile(ny, g, tau), bodies=bodies,
                  bonds=[bonds], steps=20000,
                  meta=dict(umax=umax, nu=nu, dx_um=dx_um, ar=ar, ca=ca, ncell=ncell, n_bound0=20,
                            cell_types=types))


def config_c3(seed=0, members=256):
    """The batched ensemble: `members` independent capillaries (c3_member)."""
    return [c3_member(seed, k) for k in range(members)]


def config_ensemble_small():
    """Four small members of one ensemble for parity tests: ragged widths
    (37, 64, 100, 131), 24 rows (a multiple of the tile height); a cell and
    a bonded particle, a lone cell, a cell and particle again with other
    seeds, and an empty channel."""
    return [config_tiny(nx=37, ny=24, seed=3),
            config_tiny(nx=64, ny=24, seed=4, kinds=(DEFORMABLE,)),
            config_tiny(nx=100, ny=24, seed=5),
            config_tiny(nx=131, ny=24, seed=6, kinds=())]


def config_tiny(nx=37, ny=22, tau=0.8, seed=3, walls=3, kinds=(DEFORMABLE, RIGID), umax=2e-3, ca=5e-2):
    """Small channel that still spans several kernel tiles with ragged edges:
    a deformable circle and an adhered particle with bonds, parameters scaled
    up so that the coupling terms are far above round-off in a few hundred
    steps."""
    nu = viscosity(tau)
    g = 8.0 * nu * umax / ny ** 2 if walls else 1e-6
    ks = stiffness(umax, tau, ca)
    bodies = []
    bonds = []
    cy = (ny - 1) / 2.0
    if DEFORMABLE in kinds:
        bodies.append(Body(DEFORMABLE, circle(40, 5.0, 9.3, cy + 0.37), None, ks=ks, kb=0.1 * ks,
                           rho_r=1.0, tag=TAG_CELL))
    ycr = 0.6
    yeq = 0.3
    if RIGID in kinds or FIXED in kinds:
        kind = RIGID if RIGID in kinds else FIXED
        pxy = ellipse(24, 4.0, 1.5, 24.6, -0.5 + yeq + 1.5)
        bodies.append(Body(kind, pxy, None, rho_r=1.1, tag=TAG_PARTICLE))
        if walls:
            host, frac = place_sites(pxy, 10, ycr)
            bonds.append(Bonds(len(bodies) - 1, host, frac, sigma=2e-3, ycr=ycr, yeq=yeq, kf=0.05,
                               kr0=2e-3, lb=ycr / 6.0, seed=seed))
    ux = poiseuille_profile(ny, g, tau) if walls else None
    return Config(f"tiny_{nx}x{ny}", nx, ny, tau, g, walls=walls, ux_init=ux, bodies=bodies, bonds=bonds,
                  meta=dict(umax=umax, nu=nu))


def config_contact(nx=48, ny=24, tau=0.8, gap=0.55, rep_pref=2e-4, n=24, R=4.0, kinds=(DEFORMABLE, RIGID)):
    """Two bodies closer than the repulsion range (Eq. 12) in a channel at
    rest: the vertex at angle 0 of the first and the vertex at angle pi of
    the second are gap apart, so a handful of vertex pairs interact.  The
    prefactor is raised so that the repulsion dominates the round-off."""
    ks = stiffness(1e-3, tau, 5e-2)
    cy = (ny - 1) / 2.0 + 0.31
    xa = 0.5 * nx - R - 0.5 * gap
    bodies = []
    for k, (kind, cx) in enumerate(zip(kinds, (xa, xa + 2 * R + gap))):
        xy = circle(n, R, cx, cy, start=0.0)
        if kind == DEFORMABLE:
            bodies.append(Body(DEFORMABLE, xy, None, ks=ks, kb=0.1 * ks, rho_r=1.0, tag=TAG_CELL))
        else:
            bodies.append(Body(kind, xy, None, rho_r=1.1, tag=TAG_PARTICLE))
    return Config(f"contact_{nx}x{ny}", nx, ny, tau, 0.0, walls=3, ux_init=None, bodies=bodies,
                  rep_pref=rep_pref, meta=dict(gap=gap))


def lattice_only(nx, ny, tau, walls=3, umax=1e-3, seed=0, noise=0.0):
    """Channel without bodies; optionally a seeded perturbation of the initial
    velocity (returned as a per-node array in meta['ux0'], meta['uy0'])."""
    nu = viscosity(tau)
    g = 8.0 * nu * umax / ny ** 2 if walls else 1e-6
    cfg = Config(f"lattice_{nx}x{ny}", nx, ny, tau, g, walls=walls,
                 ux_init=poiseuille_profile(ny, g, tau) if walls else None, meta=dict(umax=umax))
    return cfg


def tube3d_params(re=0.01, nx=256, diameter=64, tau=1.0):
    """The 3D extension's tube: D3Q19, a circular tube of the given diameter
    (nodes) and length nx along x, tau = 1, driven by the body force that
    gives Hagen-Poiseuille flow at Reynolds number re = u_mean D / nu
    (u_mean = g R^2 / (8 nu))."""
    nu = (tau - 0.5) / 3.0
    R = diameter / 2.0
    u_mean = re * nu / diameter
    g = 8.0 * nu * u_mean / (R * R)
    return dict(nx=nx, ny=diameter, nz=diameter, tau=tau, gx=g, radius=R, u_mean=u_mean)


CELL_3D = dict(gs=5e-3, c=1.0, ka=0.05, kv=0.05, mass=1.0, kb=2e-3)
PARTICLE_3D = dict(gs=5e-2, c=1.0, ka=0.5, kv=0.5, mass=1.0, kb=2e-2)
BONDS_3D = dict(sigma=1e-3, yeq=1.0, ycr=3.0, kf=0.05, kr0=0.005, lb=1.0, seed=2)


def tube3d_workload(p=None, sites=300, seed=21):
    """The 3D extension's workload in the tube of tube3d_params(): four
    2562-vertex oblate cells (radius 8, axes 1, 1, 0.5) off the axis, and a
    642-vertex oblate particle (radius 4, axes 1, 1, 0.5, its flat side 2.5
    nodes from the wall) carrying `sites` ligand sites at seeded random
    triangles and barycentric points.  Returns a dict: cells [(xyz, tri)],
    particle (xyz, tri), sites (tri [n], bary [n][2]), and the constants
    CELL_3D, PARTICLE_3D, BONDS_3D."""
    p = p or tube3d_params()
    c = 0.5 * (p["ny"] - 1)
    cells = [icosphere(4, 8.0, (40.2 + 60 * k, c + (9.0, -7.5, 4.0, -10.0)[k], c + (2.0, 8.0, -9.0, -1.5)[k]),
                       axes=(1.0, 1.0, 0.5)) for k in range(4)]
    part = icosphere(3, 4.0, (128.7, c + 0.3, c - (p["radius"] - 4.5)), axes=(1.0, 1.0, 0.5))
    rng = np.random.default_rng(seed)
    st = rng.integers(0, len(part[1]), sites).astype(np.int32)
    u = rng.random((sites, 2))
    u[u.sum(axis=1) > 1] = 1 - u[u.sum(axis=1) > 1]
    return dict(cells=cells, particle=part, sites=(st, u), cell=CELL_3D, part=PARTICLE_3D, bonds=BONDS_3D)


def icosphere(level, radius=1.0, center=(0.0, 0.0, 0.0), axes=(1.0, 1.0, 1.0)):
    """A triangulated sphere: the icosahedron with every triangle split in
    four `level` times, vertices pushed to the sphere, then scaled by axes
    (an oblate body for axes like (1, 1, 0.5)) and placed at center.  Level
    3: 642 vertices and 1280 triangles; level 4: 2562 and 5120.  Triangles
    are counter-clockwise seen from outside.  Returns (xyz [nv][3], tri
    [nt][3])."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    tris = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
            (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
            (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                mid[key] = len(verts) - 1
            return mid[key]
        new = []
        for a, b, c in tris:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            new += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        tris = new
    xyz = np.array(verts) * np.asarray(axes, dtype=np.float64) * radius + np.asarray(center, dtype=np.float64)
    return xyz, np.array(tris, dtype=np.int32)
