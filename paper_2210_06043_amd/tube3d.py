"""ctypes binding of the 3D extension's lattice (``include/capib3d.h``):
D3Q19 BGK with the Guo term in a capillary tube, in ``libcapib.so``.

Argument marshalling only; every step runs in the library's kernels.  torch
provides the device workspace and the stream.
"""
import ctypes as C

import numpy as np

from . import capib

TUBE, SLAB, BOX = 0, 1, 2
Q = 19
_P = C.c_void_p
_dp = C.POINTER(C.c_double)


class capib3d_lattice(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("tau", C.c_double), ("gx", C.c_double),
                ("geometry", C.c_int32), ("radius", C.c_double), ("storage", C.c_int32), ("fp16_scale", C.c_double),
                ("max_vertices", C.c_int32), ("max_membranes", C.c_int32), ("max_membrane_vertices", C.c_int32),
                ("max_membrane_triangles", C.c_int32), ("max_sites", C.c_int32)]


class capib3d_bonds(C.Structure):
    _fields_ = [("sigma", C.c_double), ("yeq", C.c_double), ("ycr", C.c_double), ("kf", C.c_double), ("kr0", C.c_double),
                ("lb", C.c_double), ("seed", C.c_uint64)]


class capib3d_membrane(C.Structure):
    _fields_ = [("gs", C.c_double), ("c", C.c_double), ("ka", C.c_double), ("kv", C.c_double), ("mass", C.c_double),
                ("kb", C.c_double)]


SIGNATURES = {
    "capib3d_create": (C.c_int, [C.POINTER(capib3d_lattice), _P, C.POINTER(_P)]),
    "capib3d_destroy": (None, [_P]),
    "capib3d_workspace_bytes": (C.c_size_t, [_P]),
    "capib3d_bind_workspace": (C.c_int, [_P, _P, C.c_size_t]),
    "capib3d_init_flow": (C.c_int, [_P, _dp]),
    "capib3d_add_fixed_body": (C.c_int, [_P, C.c_int32, _dp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "capib3d_body_forces": (C.c_int, [_P, _dp]),
    "capib3d_vertices": (C.c_int32, [_P]),
    "capib3d_set_ib_schedule": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "capib3d_add_membrane": (C.c_int, [_P, C.c_int32, _dp, C.c_int32, C.POINTER(C.c_int32), C.c_void_p,
                                       C.POINTER(C.c_int32)]),
    "capib3d_read_membrane_vertices": (C.c_int, [_P, _dp]),
    "capib3d_write_membrane_vertices": (C.c_int, [_P, _dp]),
    "capib3d_membrane_spread_forces": (C.c_int, [_P, _dp]),
    "capib3d_membrane_totals": (C.c_int, [_P, C.c_int32, _dp]),
    "capib3d_error_flags": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "capib3d_add_bonds": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_int32), _dp, C.c_void_p]),
    "capib3d_read_bonds": (C.c_int, [_P, C.POINTER(C.c_int32), _dp, C.POINTER(C.c_int64)]),
    "capib3d_write_bonds": (C.c_int, [_P, C.POINTER(C.c_int32), _dp]),
    "capib3d_membranes": (C.c_int32, [_P]),
    "capib3d_membrane_vertex_count": (C.c_int32, [_P]),
    "capib3d_step": (C.c_int, [_P, C.c_int32]),
    "capib3d_read_macro": (C.c_int, [_P, _dp, _dp, _dp, _dp]),
    "capib3d_read_populations": (C.c_int, [_P, _dp]),
    "capib3d_write_populations": (C.c_int, [_P, _dp]),
    "capib3d_diagnostics": (C.c_int, [_P, _dp, C.POINTER(C.c_int64)]),
    "capib3d_fluid_nodes": (C.c_int64, [_P]),
    "capib3d_last_error": (C.c_char_p, [_P]),
}
_ready = False


def _lib():
    global _ready
    L = capib.load_library()
    if not _ready:
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _ready = True
    return L


def _d(a):
    return a.ctypes.data_as(_dp)


def hagen_poiseuille(ny, nz, radius, tau, gx):
    """u(y, z) = g (R^2 - r^2) / (4 nu) inside the tube, 0 outside ([nz][ny])."""
    nu = (tau - 0.5) / 3.0
    y = np.arange(ny) - 0.5 * (ny - 1)
    z = np.arange(nz) - 0.5 * (nz - 1)
    r2 = z[:, None] ** 2 + y[None, :] ** 2
    return np.where(r2 < radius * radius, gx / (4 * nu) * (radius * radius - r2), 0.0)


def fp16_scale_for(umax, headroom=16.0):
    """Power-of-two scale for FP16 storage of the deviations: the flow speed
    maps to 65504 / headroom (as for the 2D lattice)."""
    import math
    return 2.0 ** math.floor(math.log2(65504.0 / (headroom * umax)))


class Tube3D:
    """A D3Q19 tube on the GPU (workspace allocated with torch)."""

    def __init__(self, nx, ny, nz, tau, gx, geometry=TUBE, radius=0.0, stream=None, storage=capib.FP32_SHIFTED,
                 fp16_scale=1.0, max_vertices=0, max_membranes=0, max_membrane_vertices=0, max_membrane_triangles=0,
                 max_sites=0):
        import torch
        self.torch = torch
        self.L = _lib()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        lat = capib3d_lattice(nx, ny, nz, tau, gx, geometry, radius, storage, fp16_scale, max_vertices, max_membranes,
                              max_membrane_vertices, max_membrane_triangles, max_sites)
        self.ctx = _P()
        st = self.L.capib3d_create(C.byref(lat), _P(self.stream.cuda_stream), C.byref(self.ctx))
        if st != capib.CAPIB_OK:
            raise capib.CapibError(st, "capib3d_create refused the lattice")
        self.nx, self.ny, self.nz, self.tau, self.gx = nx, ny, nz, tau, gx
        nbytes = self.L.capib3d_workspace_bytes(self.ctx)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize()
        self._check(self.L.capib3d_bind_workspace(self.ctx, _P((self.workspace.data_ptr() + 255) & ~255), nbytes))

    def _check(self, st):
        if st != capib.CAPIB_OK:
            raise capib.CapibError(st, self.L.capib3d_last_error(self.ctx).decode())

    def __del__(self):
        if getattr(self, "ctx", None):
            self.L.capib3d_destroy(self.ctx)
            self.ctx = None

    @property
    def fluid_nodes(self):
        return int(self.L.capib3d_fluid_nodes(self.ctx))

    def init_flow(self, ux_of_yz=None):
        a = None if ux_of_yz is None else np.ascontiguousarray(ux_of_yz, dtype=np.float64)
        if a is not None:
            assert a.shape == (self.nz, self.ny)
        self._check(self.L.capib3d_init_flow(self.ctx, None if a is None else _d(a)))

    def add_fixed_body(self, xyz, tri):
        """A fixed immersed body (vertices [nv][3], triangles [ntri][3]);
        returns the index of its first vertex."""
        X = np.ascontiguousarray(xyz, dtype=np.float64)
        T = np.ascontiguousarray(tri, dtype=np.int32)
        assert X.ndim == 2 and X.shape[1] == 3 and T.ndim == 2 and T.shape[1] == 3
        first = C.c_int32()
        self._check(self.L.capib3d_add_fixed_body(self.ctx, X.shape[0], _d(X), T.shape[0],
                                                  T.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(first)))
        return first.value

    @property
    def vertices(self):
        return int(self.L.capib3d_vertices(self.ctx))

    def body_forces(self):
        """Force of the last step on the fluid at every vertex, [nv][3]."""
        out = np.zeros((self.vertices, 3))
        self._check(self.L.capib3d_body_forces(self.ctx, _d(out)))
        return out

    def add_membrane(self, xyz, tri, gs, c, ka, kv, mass, kb=0.0):
        """A deformable membrane (vertices [nv][3], triangles [ntri][3]
        counter-clockwise from outside; Skalak G_s and C, area and volume
        penalties, vertex mass, bending k_b); returns its first vertex index."""
        X = np.ascontiguousarray(xyz, dtype=np.float64)
        T = np.ascontiguousarray(tri, dtype=np.int32)
        assert X.ndim == 2 and X.shape[1] == 3 and T.ndim == 2 and T.shape[1] == 3
        par = capib3d_membrane(gs, c, ka, kv, mass, kb)
        first = C.c_int32()
        self._check(self.L.capib3d_add_membrane(self.ctx, X.shape[0], _d(X), T.shape[0],
                                                T.ctypes.data_as(C.POINTER(C.c_int32)), C.cast(C.byref(par), C.c_void_p),
                                                C.byref(first)))
        return first.value

    @property
    def membranes(self):
        return int(self.L.capib3d_membranes(self.ctx))

    @property
    def membrane_vertex_count(self):
        return int(self.L.capib3d_membrane_vertex_count(self.ctx))

    def membrane_vertices(self):
        out = np.zeros((self.membrane_vertex_count, 3))
        self._check(self.L.capib3d_read_membrane_vertices(self.ctx, _d(out)))
        return out

    def set_membrane_vertices(self, X):
        X = np.ascontiguousarray(X, dtype=np.float64)
        assert X.shape == (self.membrane_vertex_count, 3)
        self._check(self.L.capib3d_write_membrane_vertices(self.ctx, _d(X)))

    def membrane_spread_forces(self):
        out = np.zeros((self.membrane_vertex_count, 3))
        self._check(self.L.capib3d_membrane_spread_forces(self.ctx, _d(out)))
        return out

    def membrane_totals(self, m):
        """(area, volume) at the start of the last step, (rest area, rest volume)"""
        out = np.zeros(4)
        self._check(self.L.capib3d_membrane_totals(self.ctx, int(m), _d(out)))
        return out

    def add_bonds(self, m, tri, bary, sigma, yeq, ycr, kf, kr0, lb, seed):
        """Bond sites on membrane m: triangle [ns] (index among its
        triangles) and barycentric weights [ns][2]; all start unbound."""
        T = np.ascontiguousarray(tri, dtype=np.int32)
        B = np.ascontiguousarray(bary, dtype=np.float64).reshape(-1, 2)
        par = capib3d_bonds(sigma, yeq, ycr, kf, kr0, lb, seed)
        self._check(self.L.capib3d_add_bonds(self.ctx, int(m), len(T), T.ctypes.data_as(C.POINTER(C.c_int32)), _d(B),
                                             C.cast(C.byref(par), C.c_void_p)))
        self.nsite = len(T)

    def bonds(self):
        """(bound [ns], anchors [ns][3], bound count)"""
        b = np.zeros(self.nsite, dtype=np.int32)
        a = np.zeros((self.nsite, 3))
        n = C.c_int64()
        self._check(self.L.capib3d_read_bonds(self.ctx, b.ctypes.data_as(C.POINTER(C.c_int32)), _d(a), C.byref(n)))
        return b, a, n.value

    def set_bonds(self, bound, anchor):
        b = np.ascontiguousarray(bound, dtype=np.int32)
        a = np.ascontiguousarray(anchor, dtype=np.float64)
        self._check(self.L.capib3d_write_bonds(self.ctx, b.ctypes.data_as(C.POINTER(C.c_int32)), _d(a)))

    def error_flags(self):
        f = C.c_int32()
        self._check(self.L.capib3d_error_flags(self.ctx, C.byref(f)))
        return f.value

    def set_ib_schedule(self, share_node_u, share_vertex):
        """Percent of the work items swept in the launch that computes the
        stencil nodes' velocities and in the one that computes the vertex
        forces (a schedule knob: the result does not depend on it)."""
        self._check(self.L.capib3d_set_ib_schedule(self.ctx, int(share_node_u), int(share_vertex)))

    def step(self, n=1):
        self._check(self.L.capib3d_step(self.ctx, int(n)))

    def synchronize(self):
        self.stream.synchronize()

    def macro(self):
        d, ux, uy, uz = (np.zeros((self.nz, self.ny, self.nx)) for _ in range(4))
        self._check(self.L.capib3d_read_macro(self.ctx, _d(d), _d(ux), _d(uy), _d(uz)))
        return d, ux, uy, uz

    def populations(self):
        out = np.zeros((Q, self.nz, self.ny, self.nx))
        self._check(self.L.capib3d_read_populations(self.ctx, _d(out)))
        return out

    def set_populations(self, A):
        A = np.ascontiguousarray(A, dtype=np.float64)
        assert A.shape == (Q, self.nz, self.ny, self.nx)
        self._check(self.L.capib3d_write_populations(self.ctx, _d(A)))

    def diagnostics(self):
        out = np.zeros(4)
        step = C.c_int64()
        self._check(self.L.capib3d_diagnostics(self.ctx, _d(out), C.byref(step)))
        return dict(mass=out[0], mom_x=out[1], mom_y=out[2], mom_z=out[3], step=step.value)
