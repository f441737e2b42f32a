"""ctypes wrapper of the FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The HIP library never imports it.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB selects another build of oracle.c (the sanitizer test loads the
# AddressSanitizer/UndefinedBehaviorSanitizer copy this way)
_LIB_PATH = os.environ.get("ORACLE_LIB", os.path.join(HERE, "liboracle.so"))
_lib = None

DEFORMABLE, RIGID, FIXED = 0, 1, 2
STEN_VELOCITY, STEN_PROBE = 0, 1

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def _d(a):
    return a.ctypes.data_as(_dp)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_interactions.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double]
        L.orc_set_velocity_wall.argtypes = [C.c_void_p, C.c_int]
        L.orc_init_flow.argtypes = [C.c_void_p, _dp]
        L.orc_get_populations.argtypes = [C.c_void_p, _dp]
        L.orc_set_populations.argtypes = [C.c_void_p, _dp]
        L.orc_get_step.restype = C.c_int64
        L.orc_get_step.argtypes = [C.c_void_p]
        L.orc_min_margin.restype = C.c_double
        L.orc_min_margin.argtypes = [C.c_void_p]
        L.orc_margins.argtypes = [C.c_void_p, _dp]
        L.orc_reset_margins.argtypes = [C.c_void_p]
        L.orc_bond_flips.restype = C.c_int64
        L.orc_bond_flips.argtypes = [C.c_void_p]
        L.orc_set_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_get_threads.argtypes = []
        L.orc_set_body_state.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
        L.orc_get_body_state.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
        L.orc_set_bonds.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_ubyte), _dp]
        L.orc_flags.restype = C.c_int
        L.orc_flags.argtypes = [C.c_void_p]
        L.orc_add_body.restype = C.c_int
        L.orc_add_body.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double,
                                   C.c_double, C.c_double, C.c_double, C.c_int]
        L.orc_add_bonds.restype = C.c_int
        L.orc_add_bonds.argtypes = [C.c_void_p, C.c_int, C.c_int, _ip, _dp, C.c_double, C.c_double,
                                    C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint64]
        L.orc_get_vertices.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc_get_bonds.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_ubyte), _dp]
        L.orc_count_bound.restype = C.c_int
        L.orc_count_bound.argtypes = [C.c_void_p, C.c_int]
        L.orc_get_body_work.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]
        L.orc_get_rigid.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc_body_diag.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_macro.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_node_fields.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp]
        L.orc_totals.argtypes = [C.c_void_p, _dp]
        L.orc_lattice_tables.argtypes = [_ip, _ip, _dp]
        L.orc_heq.argtypes = [C.c_double, C.c_double, C.c_double, _dp]
        L.orc_guo.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, _dp]
        L.orc_phi.restype = C.c_double
        L.orc_phi.argtypes = [C.c_double]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.orc_uniform.restype = C.c_double
        L.orc_uniform.argtypes = [C.c_uint64, C.c_int64, C.c_int32]
        L.orc_stencil.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, _ip, _ip, _dp]
        L.orc_interp_field.restype = C.c_double
        L.orc_interp_field.argtypes = [C.c_void_p, _dp, C.c_double, C.c_double, C.c_int]
        L.orc_polygon.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_polar_moment.restype = C.c_double
        L.orc_polar_moment.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double]
        L.orc_membrane_forces.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                          C.c_double, _dp]
        L.orc_set_body_work.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.orc_integrate_body.argtypes = [C.c_void_p, C.c_int]
        L.orc_relax_membrane.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_double, C.c_int, _dp, _dp]
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the oracle's per-node loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def threads():
    return lib().orc_get_threads()


# ---- point functions -----------------------------------------------------------

def lattice_tables():
    ex = np.zeros(9, np.int32)
    ey = np.zeros(9, np.int32)
    w = np.zeros(9)
    lib().orc_lattice_tables(ex.ctypes.data_as(_ip), ey.ctypes.data_as(_ip), _d(w))
    return ex, ey, w


def heq(drho, ux, uy):
    out = np.zeros(9)
    lib().orc_heq(drho, ux, uy, _d(out))
    return out


def guo(tau, ux, uy, Fx, Fy):
    out = np.zeros(9)
    lib().orc_guo(tau, ux, uy, Fx, Fy, _d(out))
    return out


def phi(r):
    return lib().orc_phi(float(r))


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(o[i]) for i in range(4)]


def uniform(seed, n, s):
    return lib().orc_uniform(seed, n, s)


def polygon(xy):
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    n = len(xy)
    x = np.ascontiguousarray(xy[:, 0])
    y = np.ascontiguousarray(xy[:, 1])
    out = np.zeros(4)
    th, nvx, nvy, ln, nlx, nly = (np.zeros(n) for _ in range(6))
    lib().orc_polygon(n, _d(x), _d(y), _d(out), _d(th), _d(nvx), _d(nvy), _d(ln), _d(nlx), _d(nly))
    return dict(area=out[0], perimeter=out[1], cx=out[2], cy=out[3], theta=th,
                nv=np.stack([nvx, nvy], 1), length=ln, nl=np.stack([nlx, nly], 1))


def polar_moment(xy, cx, cy):
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    x = np.ascontiguousarray(xy[:, 0])
    y = np.ascontiguousarray(xy[:, 1])
    return lib().orc_polar_moment(len(xy), _d(x), _d(y), cx, cy)


def membrane_forces(xy, xy_rest, ks, kb, ka, pref):
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    xr = np.ascontiguousarray(xy_rest, dtype=np.float64).reshape(-1)
    f = np.zeros_like(xy)
    lib().orc_membrane_forces(len(xy) // 2, _d(xy), _d(xr), ks, kb, ka, pref, _d(f))
    return f.reshape(-1, 2)


def relax_membrane(xy, xy_rest, ks, kb, ka, pref, rho_r, nsteps):
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    xr = np.ascontiguousarray(xy_rest, dtype=np.float64).reshape(-1)
    out = np.zeros_like(xy)
    hist = np.zeros(max(nsteps, 1))
    lib().orc_relax_membrane(len(xy) // 2, _d(xy), _d(xr), ks, kb, ka, pref, rho_r, nsteps, _d(out), _d(hist))
    return out.reshape(-1, 2), hist[:nsteps]


# ---- the simulation ------------------------------------------------------------

class Sim:
    """One FP64 simulation: lattice, bodies, bonds, step."""

    def __init__(self, nx, ny, tau, gx=0.0, gy=0.0, walls=3):
        self.nx, self.ny = nx, ny
        self.p = lib().orc_create(nx, ny, tau, gx, gy, walls)
        if not self.p:
            raise ValueError("oracle rejected the lattice parameters")
        self.nv = []
        self.ns = []

    def __del__(self):
        if getattr(self, "p", None):
            lib().orc_destroy(self.p)
            self.p = None

    def set_interactions(self, rep_pref, rep_cut, probe_dist):
        lib().orc_set_interactions(self.p, rep_pref, rep_cut, probe_dist)

    def set_velocity_wall(self, image):
        """Velocity coupling across a wall: odd image (True, the default) or
        rows beyond the wall as wall nodes at rest (False, the earlier reading)."""
        lib().orc_set_velocity_wall(self.p, 1 if image else 0)

    def init_flow(self, ux_of_y=None):
        if ux_of_y is None:
            lib().orc_init_flow(self.p, None)
        else:
            u = np.ascontiguousarray(ux_of_y, dtype=np.float64)
            assert u.shape == (self.ny,)
            lib().orc_init_flow(self.p, _d(u))

    def add_body(self, kind, xy, xy_rest=None, ks=0.0, kb=0.0, ka=0.0, pref=1.0 / 3.0, rho_r=1.0, tag=0):
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
        xr = None if xy_rest is None else np.ascontiguousarray(xy_rest, dtype=np.float64).reshape(-1)
        k = lib().orc_add_body(self.p, kind, len(xy) // 2, _d(xy), None if xr is None else _d(xr),
                               ks, kb, ka, pref, rho_r, tag)
        if k < 0:
            raise ValueError("oracle rejected the body")
        self.nv.append(len(xy) // 2)
        self.ns.append(0)
        return k

    def add_bonds(self, body, host, frac, sigma, ycr, yeq, kf, kr0, lb, seed):
        host = np.ascontiguousarray(host, dtype=np.int32)
        frac = np.ascontiguousarray(frac, dtype=np.float64)
        r = lib().orc_add_bonds(self.p, body, len(host), host.ctypes.data_as(_ip), _d(frac), sigma, ycr,
                                yeq, kf, kr0, lb, seed)
        if r < 0:
            raise ValueError("oracle rejected the bonds")
        self.ns[body] = len(host)

    def step(self, n=1):
        lib().orc_step(self.p, int(n))

    @property
    def n(self):
        return lib().orc_get_step(self.p)

    @property
    def min_margin(self):
        return lib().orc_min_margin(self.p)

    def margins(self):
        """(smallest |draw - P| / P of the bond decisions, smallest |gap - y_cr|
        of the formation decisions the gap decided) since the start or the
        last reset_margins()."""
        out = np.zeros(2)
        lib().orc_margins(self.p, _d(out))
        return float(out[0]), float(out[1])

    def reset_margins(self):
        """Restarts the margin minima and the flip count."""
        lib().orc_reset_margins(self.p)

    @property
    def flips(self):
        """Bond state changes (formations and ruptures) since the start or
        the last reset_margins()."""
        return lib().orc_bond_flips(self.p)

    def set_step(self, n):
        lib().orc_set_step(self.p, int(n))

    def set_body_state(self, body, xy=None, dxy_prev=None, rigid=None):
        """Overwrite x^n, x^n - x^{n-1} (deformable) and the rigid state
        {xc, yc, phi, ucx, ucy, ucx_prev, ucy_prev, omega, omega_prev}."""
        a = None if xy is None else np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
        d = None if dxy_prev is None else np.ascontiguousarray(dxy_prev, dtype=np.float64).reshape(-1)
        r = None if rigid is None else np.ascontiguousarray(rigid, dtype=np.float64).reshape(-1)
        for arr, n in ((a, 2 * self.nv[body]), (d, 2 * self.nv[body]), (r, 9)):
            assert arr is None or arr.shape == (n,)
        lib().orc_set_body_state(self.p, body, None if a is None else _d(a), None if d is None else _d(d),
                                 None if r is None else _d(r))

    def body_state(self, body):
        n = self.nv[body]
        xy, d, r = np.zeros((n, 2)), np.zeros((n, 2)), np.zeros(9)
        lib().orc_get_body_state(self.p, body, _d(xy), _d(d), _d(r))
        return dict(xy=xy, dxy_prev=d, rigid=r)

    def set_bonds(self, body, state, anchor):
        st = np.ascontiguousarray(state, dtype=np.uint8)
        an = np.ascontiguousarray(anchor, dtype=np.float64)
        assert st.shape == (self.ns[body],) and an.shape == (self.ns[body],)
        lib().orc_set_bonds(self.p, body, st.ctypes.data_as(C.POINTER(C.c_ubyte)), _d(an))

    @property
    def flags(self):
        return lib().orc_flags(self.p)

    def populations(self):
        out = np.zeros((9, self.ny, self.nx))
        lib().orc_get_populations(self.p, _d(out))
        return out

    def set_populations(self, A):
        A = np.ascontiguousarray(A, dtype=np.float64)
        assert A.shape == (9, self.ny, self.nx)
        lib().orc_set_populations(self.p, _d(A))

    def macro(self):
        r, ux, uy = (np.zeros((self.ny, self.nx)) for _ in range(3))
        lib().orc_macro(self.p, _d(r), _d(ux), _d(uy))
        return r, ux, uy

    def node_fields(self):
        out = [np.zeros((self.ny, self.nx)) for _ in range(5)]
        lib().orc_node_fields(self.p, *[_d(a) for a in out])
        return dict(sxx=out[0], sxy=out[1], syy=out[2], fibx=out[3], fiby=out[4])

    def totals(self):
        out = np.zeros(3)
        lib().orc_totals(self.p, _d(out))
        return out

    def vertices(self, body):
        out = np.zeros((self.nv[body], 2))
        lib().orc_get_vertices(self.p, body, _d(out))
        return out

    def bonds(self, body):
        ns = self.ns[body]
        st = np.zeros(ns, np.uint8)
        an = np.zeros(ns)
        lib().orc_get_bonds(self.p, body, st.ctypes.data_as(C.POINTER(C.c_ubyte)), _d(an))
        return st, an

    def count_bound(self, body):
        return lib().orc_count_bound(self.p, body)

    def body_work(self, body):
        n = self.nv[body]
        us, pr, f, U = np.zeros((n, 2)), np.zeros((n, 4)), np.zeros((n, 2)), np.zeros((n, 2))
        lib().orc_get_body_work(self.p, body, _d(us), _d(pr), _d(f), _d(U))
        return dict(ustar=us, probe=pr, force=f, U=U)

    def rigid(self, body):
        o = np.zeros(8)
        lib().orc_get_rigid(self.p, body, _d(o))
        return dict(xc=o[0], yc=o[1], phi=o[2], ucx=o[3], ucy=o[4], om=o[5], mass=o[6], inertia=o[7])

    def body_diag(self, body):
        o = np.zeros(8)
        lib().orc_body_diag(self.p, body, _d(o))
        return dict(area=o[0], perimeter=o[1], cx=o[2], cy=o[3], A0=o[4], P0=o[5], n_bound=int(o[6]),
                    vmass=o[7])

    def set_body_work(self, body, ustar=None, force=None):
        us = None if ustar is None else np.ascontiguousarray(ustar, dtype=np.float64).reshape(-1)
        f = None if force is None else np.ascontiguousarray(force, dtype=np.float64).reshape(-1)
        lib().orc_set_body_work(self.p, body, None if us is None else _d(us), None if f is None else _d(f))

    def integrate_body(self, body):
        lib().orc_integrate_body(self.p, body)

    def stencil(self, X, Y, mode=STEN_VELOCITY):
        ii = np.zeros(4, np.int32)
        jj = np.zeros(4, np.int32)
        w = np.zeros(16)
        lib().orc_stencil(self.p, X, Y, mode, ii.ctypes.data_as(_ip), jj.ctypes.data_as(_ip), _d(w))
        return ii, jj, w.reshape(4, 4)

    def interp_field(self, field, X, Y, mode=STEN_VELOCITY):
        f = np.ascontiguousarray(field, dtype=np.float64)
        assert f.shape == (self.ny, self.nx)
        return lib().orc_interp_field(self.p, _d(f), X, Y, mode)
