"""ctypes wrapper of the FP64 oracle of the 3D extension's lattice
(``oracle/oracle3d.c``): D3Q19 BGK with the Guo term in a capillary tube.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the CPU-baseline leg of
``bench.py``.  The HIP library never imports it.
"""
import ctypes as C

import numpy as np

from . import lib as _lib

TUBE, SLAB, BOX = 0, 1, 2
_dp = C.POINTER(C.c_double)
_ready = False


def _d(a):
    return a.ctypes.data_as(_dp)


def _L():
    global _ready
    L = _lib()
    if not _ready:
        L.orc3_create.restype = C.c_void_p
        L.orc3_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_double]
        L.orc3_destroy.argtypes = [C.c_void_p]
        L.orc3_is_fluid.restype = C.c_int
        L.orc3_is_fluid.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc3_init_flow.argtypes = [C.c_void_p, _dp]
        L.orc3_get_populations.argtypes = [C.c_void_p, _dp]
        L.orc3_set_populations.argtypes = [C.c_void_p, _dp]
        L.orc3_get_step.restype = C.c_longlong
        L.orc3_get_step.argtypes = [C.c_void_p]
        L.orc3_step.argtypes = [C.c_void_p, C.c_int]
        L.orc3_macro.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.orc3_totals.argtypes = [C.c_void_p, _dp]
        L.orc3_lattice_tables.argtypes = [C.POINTER(C.c_int), _dp]
        L.orc3_heq.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _dp]
        L.orc3_guo.argtypes = [C.c_double] + [C.c_double] * 6 + [_dp]
        L.orc3_add_fixed_body.restype = C.c_int
        L.orc3_add_fixed_body.argtypes = [C.c_void_p, C.c_int, _dp, C.c_int, C.POINTER(C.c_int)]
        L.orc3_ib_force.argtypes = [C.c_void_p, _dp]
        L.orc3_vertex_weights.argtypes = [C.c_void_p, _dp]
        L.orc3_add_membrane.restype = C.c_int
        L.orc3_add_membrane.argtypes = [C.c_void_p, C.c_int, _dp, C.c_int, C.POINTER(C.c_int)] + [C.c_double] * 6
        L.orc3_membrane_vertices.argtypes = [C.c_void_p, _dp]
        L.orc3_membrane_set_vertices.argtypes = [C.c_void_p, _dp]
        L.orc3_membrane_forces.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc3_membrane_spread_forces.argtypes = [C.c_void_p, _dp]
        L.orc3_membrane_totals.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc3_membrane_energy.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc3_add_bonds.restype = C.c_int
        L.orc3_add_bonds.argtypes = [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_int), _dp] + [C.c_double] * 6 + [
            C.c_uint64]
        L.orc3_bonds.restype = C.c_int
        L.orc3_bonds.argtypes = [C.c_void_p, C.POINTER(C.c_int), _dp]
        L.orc3_set_bonds.argtypes = [C.c_void_p, C.POINTER(C.c_int), _dp]
        L.orc3_bond_margins.argtypes = [C.c_void_p, _dp]
        L.orc3_membrane_dihedrals.restype = C.c_int
        L.orc3_membrane_dihedrals.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        _ready = True
    return L


def lattice_tables():
    e = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    _L().orc3_lattice_tables(e.ctypes.data_as(C.POINTER(C.c_int)), _d(w))
    return e.reshape(19, 3), w


def heq(drho, ux, uy, uz):
    out = np.zeros(19)
    _L().orc3_heq(drho, ux, uy, uz, _d(out))
    return out


def guo(tau, u, F):
    out = np.zeros(19)
    _L().orc3_guo(tau, u[0], u[1], u[2], F[0], F[1], F[2], _d(out))
    return out


class Tube:
    """D3Q19 lattice nx x ny x nz (x along the tube), FP64."""

    def __init__(self, nx, ny, nz, tau, gx, geom=TUBE, radius=0.0):
        self.L = _L()
        self.p = self.L.orc3_create(nx, ny, nz, tau, gx, geom, radius)
        if not self.p:
            raise ValueError("orc3_create refused the lattice")
        self.nx, self.ny, self.nz = nx, ny, nz

    def __del__(self):
        if getattr(self, "p", None):
            self.L.orc3_destroy(self.p)
            self.p = None

    def fluid(self):
        return np.array([[self.L.orc3_is_fluid(self.p, y, z) for y in range(self.ny)] for z in range(self.nz)],
                        dtype=bool)

    def init_flow(self, ux_of_yz=None):
        a = None if ux_of_yz is None else np.ascontiguousarray(ux_of_yz, dtype=np.float64)
        self.L.orc3_init_flow(self.p, None if a is None else _d(a))

    def populations(self):
        out = np.zeros((19, self.nz, self.ny, self.nx))
        self.L.orc3_get_populations(self.p, _d(out))
        return out

    def set_populations(self, A):
        A = np.ascontiguousarray(A, dtype=np.float64)
        assert A.shape == (19, self.nz, self.ny, self.nx)
        self.L.orc3_set_populations(self.p, _d(A))

    def step(self, n=1):
        self.L.orc3_step(self.p, int(n))

    @property
    def n(self):
        return self.L.orc3_get_step(self.p)

    def macro(self):
        d, ux, uy, uz = (np.zeros((self.nz, self.ny, self.nx)) for _ in range(4))
        self.L.orc3_macro(self.p, _d(d), _d(ux), _d(uy), _d(uz))
        return d, ux, uy, uz

    def totals(self):
        out = np.zeros(4)
        self.L.orc3_totals(self.p, _d(out))
        return out

    def add_fixed_body(self, xyz, tri):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
        v0 = self.L.orc3_add_fixed_body(self.p, len(xyz), _d(xyz), len(tri),
                                        tri.ctypes.data_as(C.POINTER(C.c_int)))
        if v0 < 0:
            raise ValueError("a stencil node of the body is solid or outside the cross-section")
        self.nv = getattr(self, "nv", 0) + len(xyz)
        return v0

    def ib_force(self):
        out = np.zeros((3, self.nz, self.ny, self.nx))
        self.L.orc3_ib_force(self.p, _d(out))
        return out

    def vertex_weights(self):
        out = np.zeros(getattr(self, "nv", 0))
        self.L.orc3_vertex_weights(self.p, _d(out))
        return out

    # deformable membranes
    def add_membrane(self, xyz, tri, gs, c, ka, kv, mass, kb=0.0):
        """A closed triangulated membrane (Skalak G_s, C; area and volume
        penalties k_A, k_V; vertex mass; bending k_b); returns its first
        vertex index among the membrane vertices."""
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
        v0 = self.L.orc3_add_membrane(self.p, len(xyz), _d(xyz), len(tri), tri.ctypes.data_as(C.POINTER(C.c_int)),
                                      gs, c, ka, kv, mass, kb)
        if v0 < 0:
            raise ValueError("a stencil node of the membrane is solid or outside the cross-section")
        self.mv = getattr(self, "mv", 0) + len(xyz)
        self.mranges = getattr(self, "mranges", []) + [(v0, len(xyz))]
        return v0

    def membrane_vertices(self):
        out = np.zeros((getattr(self, "mv", 0), 3))
        self.L.orc3_membrane_vertices(self.p, _d(out))
        return out

    def set_membrane_vertices(self, X):
        X = np.ascontiguousarray(X, dtype=np.float64)
        assert X.shape == (self.mv, 3)
        self.L.orc3_membrane_set_vertices(self.p, _d(X))

    def membrane_forces(self, m):
        out = np.zeros((self.mranges[m][1], 3))
        self.L.orc3_membrane_forces(self.p, m, _d(out))
        return out

    def membrane_spread_forces(self):
        out = np.zeros((getattr(self, "mv", 0), 3))
        self.L.orc3_membrane_spread_forces(self.p, _d(out))
        return out

    def membrane_totals(self, m):
        """(area, volume, rest area, rest volume)"""
        out = np.zeros(4)
        self.L.orc3_membrane_totals(self.p, m, _d(out))
        return out

    def membrane_energy(self, m):
        """(Skalak, area penalty, volume penalty, bending)"""
        out = np.zeros(4)
        self.L.orc3_membrane_energy(self.p, m, _d(out))
        return out

    def membrane_dihedrals(self, m):
        """(current, rest) dihedral angle of every interior edge of membrane m"""
        n = self.L.orc3_membrane_dihedrals(self.p, m, None, None)
        th, th0 = np.zeros(n), np.zeros(n)
        self.L.orc3_membrane_dihedrals(self.p, m, _d(th), _d(th0))
        return th, th0

    # bonds
    def add_bonds(self, m, tri, bary, sigma, yeq, ycr, kf, kr0, lb, seed):
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        bary = np.ascontiguousarray(bary, dtype=np.float64).reshape(-1, 2)
        if self.L.orc3_add_bonds(self.p, m, len(tri), tri.ctypes.data_as(C.POINTER(C.c_int)), _d(bary), sigma, yeq, ycr,
                                 kf, kr0, lb, seed) != 0:
            raise ValueError("orc3_add_bonds refused the sites")
        self.ns = len(tri)

    def bonds(self):
        """(bound [ns], anchors [ns][3], bound count)"""
        b = np.zeros(self.ns, dtype=np.int32)
        a = np.zeros((self.ns, 3))
        n = self.L.orc3_bonds(self.p, b.ctypes.data_as(C.POINTER(C.c_int)), _d(a))
        return b, a, n

    def set_bonds(self, bound, anchor):
        b = np.ascontiguousarray(bound, dtype=np.int32)
        a = np.ascontiguousarray(anchor, dtype=np.float64)
        self.L.orc3_set_bonds(self.p, b.ctypes.data_as(C.POINTER(C.c_int)), _d(a))

    def bond_margins(self):
        out = np.zeros(3)
        self.L.orc3_bond_margins(self.p, _d(out))
        return out
