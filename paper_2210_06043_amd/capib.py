"""Thin ctypes binding of libcapib (C-ABI in include/capib.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch provides the device workspace and the stream.  There
is no fallback: if the library is missing or no GPU is present, construction
raises.
"""
import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcapib.so")

CAPIB_OK, CAPIB_E_ARG, CAPIB_E_STATE, CAPIB_E_HIP, CAPIB_E_UNSTABLE, CAPIB_E_CAPACITY = 0, -1, -2, -3, -4, -5
FP32_SHIFTED, FP16_SHIFTED = 0, 1
DEFORMABLE, RIGID, FIXED = 0, 1, 2
FLAG_VERTEX_OUT, FLAG_FLUID, FLAG_NONFINITE_IB = 1, 2, 8

_dp = C.POINTER(C.c_double)


class capib_lattice(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("tau", C.c_double), ("gx", C.c_double),
                ("gy", C.c_double), ("walls", C.c_int32), ("storage", C.c_int32), ("fp16_scale", C.c_double),
                ("max_bodies", C.c_int32), ("max_vertices", C.c_int32), ("max_sites", C.c_int32)]


class capib_membrane(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("xy", _dp), ("xy_rest", _dp), ("ks", C.c_double),
                ("kb", C.c_double), ("ka", C.c_double), ("p_ref", C.c_double), ("density_ratio", C.c_double),
                ("tag", C.c_int32), ("band", C.c_int32)]


class capib_bonds(C.Structure):
    _fields_ = [("n_sites", C.c_int32), ("host_elem", C.POINTER(C.c_int32)), ("frac", _dp),
                ("sigma", C.c_double), ("y_cr", C.c_double), ("y_eq", C.c_double), ("k_f", C.c_double),
                ("k_r0", C.c_double), ("bell_len", C.c_double), ("seed", C.c_uint64)]


class capib_diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("error_flags", C.c_int32), ("n_bodies", C.c_int32), ("mass", C.c_double),
                ("mom_x", C.c_double), ("mom_y", C.c_double), ("near_tiles", C.c_int32), ("tiles", C.c_int32)]


class capib_body_diag(C.Structure):
    _fields_ = [("area", C.c_double), ("perimeter", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("area0", C.c_double), ("perimeter0", C.c_double), ("n_bound", C.c_int32), ("kind", C.c_int32),
                ("xc", C.c_double), ("yc", C.c_double), ("phi", C.c_double), ("ucx", C.c_double),
                ("ucy", C.c_double), ("omega", C.c_double), ("n_bound0", C.c_int32), ("reserved", C.c_int32)]


class capib_tuning(C.Structure):
    _fields_ = [("split", C.c_int32), ("far_share_pct", C.c_int32), ("mark_pairs", C.c_int32),
                ("membrane_class", C.c_int32)]


_P = C.c_void_p
SIGNATURES = {
    "capib_create": (C.c_int, [C.POINTER(capib_lattice), _P, C.POINTER(_P)]),
    "capib_create_ensemble": (C.c_int, [C.POINTER(capib_lattice), C.c_int32, C.POINTER(C.c_int32), _P,
                                        C.POINTER(_P)]),
    "capib_workspace_bytes": (C.c_size_t, [_P]),
    "capib_bind_workspace": (C.c_int, [_P, _P, C.c_size_t]),
    "capib_init_flow": (C.c_int, [_P, _dp]),
    "capib_write_populations": (C.c_int, [_P, _dp]),
    "capib_read_populations": (C.c_int, [_P, _dp]),
    "capib_add_membrane": (C.c_int, [_P, C.POINTER(capib_membrane), C.POINTER(C.c_int32)]),
    "capib_add_bonds": (C.c_int, [_P, C.c_int32, C.POINTER(capib_bonds)]),
    "capib_set_interactions": (C.c_int, [_P, C.c_double, C.c_double, C.c_double]),
    "capib_step": (C.c_int, [_P, C.c_int32]),
    "capib_set_graph": (C.c_int, [_P, C.c_int32]),
    "capib_set_tuning": (C.c_int, [_P, C.POINTER(capib_tuning)]),
    "capib_get_tuning": (C.c_int, [_P, C.POINTER(capib_tuning)]),
    "capib_autotune": (C.c_int, [_P, C.c_int32, C.c_char_p, C.POINTER(capib_tuning), _dp]),
    "capib_read_macro": (C.c_int, [_P, _dp, _dp, _dp]),
    "capib_read_vertices": (C.c_int, [_P, C.c_int32, _dp]),
    "capib_read_bonds": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_uint8), _dp]),
    "capib_read_body_work": (C.c_int, [_P, C.c_int32, _dp, _dp, _dp, _dp]),
    "capib_diagnostics": (C.c_int, [_P, C.POINTER(capib_diag)]),
    "capib_body_diagnostics": (C.c_int, [_P, C.c_int32, C.POINTER(capib_body_diag)]),
    "capib_readout": (C.c_int, [_P, C.c_int32, C.c_int32, _dp]),
    "capib_read_body_state": (C.c_int, [_P, C.c_int32, _dp, _dp, _dp]),
    "capib_copy_bandwidth": (C.c_int, [_P, _P, C.c_size_t, _P]),
    "capib_diagnostics_noalloc": (C.c_int, [_P, C.POINTER(capib_diag)]),
    "capib_save": (C.c_int, [_P, _P, C.POINTER(C.c_size_t)]),
    "capib_load": (C.c_int, [_P, _P, C.c_size_t]),
    "capib_set_timing": (C.c_int, [_P, C.c_int32]),
    "capib_read_timing": (C.c_int, [_P, _dp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "capib_sample_members": (C.c_int, [_P, C.c_int32, C.c_int32, _P]),
    "capib_last_error": (C.c_char_p, [_P]),
    "capib_destroy": (None, [_P]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Loads libcapib.so (raises if it has not been built).  torch is
    imported first: its HIP runtime is then the one the library binds to,
    so that one runtime serves both (the library loaded first would bring
    in the system's copy, and torch could not initialise the device)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (see above)
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with paper_2210_06043_amd/build.py")
        L = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class CapibError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"capib status {status}: {msg}")
        self.status = status


def _d(a):
    return None if a is None else a.ctypes.data_as(_dp)


class Simulation:
    """One LBM-IB simulation on the current CUDA (HIP) device, or an ensemble
    of independent capillaries of ny rows and widths `bands` advanced
    together (nx is then ignored; fields are the stack of the members)."""

    def __init__(self, nx, ny, tau, gx=0.0, gy=0.0, walls=3, storage=FP32_SHIFTED, fp16_scale=1.0,
                 max_bodies=8, max_vertices=4096, max_sites=4096, stream=None, device=None, bands=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the capib path runs only on the GPU")
        self.L = load_library()
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        lat = capib_lattice(nx, ny, tau, gx, gy, walls, storage, fp16_scale, max_bodies, max_vertices, max_sites)
        self.ctx = _P()
        if bands is None:
            st = self.L.capib_create(C.byref(lat), _P(self.stream.cuda_stream), C.byref(self.ctx))
            self.bands = [nx]
            self.nx, self.ny = nx, ny
        else:
            w = (C.c_int32 * len(bands))(*[int(b) for b in bands])
            st = self.L.capib_create_ensemble(C.byref(lat), len(bands), w, _P(self.stream.cuda_stream),
                                              C.byref(self.ctx))
            self.bands = [int(b) for b in bands]
            self.nx, self.ny = max(self.bands), ny * len(self.bands)
        if st != CAPIB_OK:
            raise CapibError(st, "capib_create rejected the lattice")
        self.band_rows = ny
        nbytes = self.L.capib_workspace_bytes(self.ctx)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.workspace.data_ptr()
        self._ws_ptr = (ptr + 255) & ~255
        self._check(self.L.capib_bind_workspace(self.ctx, _P(self._ws_ptr), nbytes))
        self.nv = []
        self.ns = []

    def _check(self, st):
        if st != CAPIB_OK:
            raise CapibError(st, self.L.capib_last_error(self.ctx).decode())
        return st

    def close(self):
        if getattr(self, "ctx", None):
            self.L.capib_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- set-up ----------------------------------------------------------------------
    def init_flow(self, ux_of_y=None):
        u = None if ux_of_y is None else np.ascontiguousarray(ux_of_y, dtype=np.float64)
        if u is not None and u.shape != (self.band_rows,):
            raise ValueError("ux_of_y needs one value per row of a member")
        self._check(self.L.capib_init_flow(self.ctx, _d(u)))

    def write_populations(self, h):
        h = np.ascontiguousarray(h, dtype=np.float64)
        if h.shape != (9, self.ny, self.nx):
            raise ValueError("populations must be (9, ny, nx)")
        self._check(self.L.capib_write_populations(self.ctx, _d(h)))

    def read_populations(self):
        out = np.zeros((9, self.ny, self.nx))
        self._check(self.L.capib_read_populations(self.ctx, _d(out)))
        return out

    def add_membrane(self, kind, xy, xy_rest=None, ks=0.0, kb=0.0, ka=0.0, p_ref=1.0 / 3.0, density_ratio=1.0,
                     tag=0, band=0):
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
        xr = None if xy_rest is None else np.ascontiguousarray(xy_rest, dtype=np.float64).reshape(-1)
        m = capib_membrane(kind, len(xy) // 2, _d(xy), _d(xr), ks, kb, ka, p_ref, density_ratio, tag, band)
        bid = C.c_int32()
        self._check(self.L.capib_add_membrane(self.ctx, C.byref(m), C.byref(bid)))
        self.nv.append(len(xy) // 2)
        self.ns.append(0)
        return bid.value

    def add_bonds(self, body, host, frac, sigma, y_cr, y_eq, k_f, k_r0, bell_len, seed):
        host = np.ascontiguousarray(host, dtype=np.int32)
        frac = np.ascontiguousarray(frac, dtype=np.float64)
        b = capib_bonds(len(host), host.ctypes.data_as(C.POINTER(C.c_int32)), _d(frac), sigma, y_cr, y_eq, k_f,
                        k_r0, bell_len, seed)
        self._check(self.L.capib_add_bonds(self.ctx, body, C.byref(b)))
        self.ns[body] = len(host)

    def set_interactions(self, rep_prefactor, rep_cutoff, probe_dist):
        self._check(self.L.capib_set_interactions(self.ctx, rep_prefactor, rep_cutoff, probe_dist))

    # ---- stepping ----------------------------------------------------------------------
    def step(self, nsteps=1):
        self._check(self.L.capib_step(self.ctx, int(nsteps)))

    def set_graph(self, enable=True):
        self._check(self.L.capib_set_graph(self.ctx, 1 if enable else 0))

    def set_tuning(self, split=-1, far_share_pct=-1, mark_pairs=-1, membrane_class=-1):
        t = capib_tuning(split, far_share_pct, mark_pairs, membrane_class)
        self._check(self.L.capib_set_tuning(self.ctx, C.byref(t)))

    def tuning(self):
        t = capib_tuning()
        self._check(self.L.capib_get_tuning(self.ctx, C.byref(t)))
        return {k: getattr(t, k) for k, _ in capib_tuning._fields_}

    def autotune(self, steps_per_trial=200, cache_path=None):
        """Times launch configurations on this workload, applies the fastest
        (state unchanged); returns it with its ms per step."""
        t = capib_tuning()
        ms = C.c_double()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(self.L.capib_autotune(self.ctx, int(steps_per_trial), path, C.byref(t), C.byref(ms)))
        out = {k: getattr(t, k) for k, _ in capib_tuning._fields_}
        out["ms_per_step"] = ms.value
        return out

    def set_timing(self, enable=True):
        self._check(self.L.capib_set_timing(self.ctx, 1 if enable else 0))

    def read_timing(self):
        """Summed ms of the {interpolation, membrane, far-tile, sweep} launches,
        the number of steps timed and the lattice nodes each launch swept."""
        ms = np.zeros(4)
        nodes = np.zeros(4, dtype=np.int64)
        n = C.c_int64()
        self._check(self.L.capib_read_timing(self.ctx, _d(ms), C.byref(n),
                                             nodes.ctypes.data_as(C.POINTER(C.c_int64))))
        return ms, n.value, nodes

    def synchronize(self):
        self.stream.synchronize()

    # ---- read-out ----------------------------------------------------------------------
    def macro(self):
        r, ux, uy = (np.zeros((self.ny, self.nx)) for _ in range(3))
        self._check(self.L.capib_read_macro(self.ctx, _d(r), _d(ux), _d(uy)))
        return r, ux, uy

    def vertices(self, body):
        out = np.zeros((self.nv[body], 2))
        self._check(self.L.capib_read_vertices(self.ctx, body, _d(out)))
        return out

    def bonds(self, body):
        ns = self.ns[body]
        st = np.zeros(ns, np.uint8)
        an = np.zeros(ns)
        self._check(self.L.capib_read_bonds(self.ctx, body, st.ctypes.data_as(C.POINTER(C.c_uint8)), _d(an)))
        return st, an

    def body_work(self, body):
        n = self.nv[body]
        us, pr, f, U = np.zeros((n, 2)), np.zeros((n, 4)), np.zeros((n, 2)), np.zeros((n, 2))
        self._check(self.L.capib_read_body_work(self.ctx, body, _d(us), _d(pr), _d(f), _d(U)))
        return dict(ustar=us, probe=pr, force=f, U=U)

    def diagnostics(self, allow_unstable=False, noalloc=False):
        """capib_diagnostics (or, with noalloc, capib_diagnostics_noalloc)."""
        d = capib_diag()
        fn = self.L.capib_diagnostics_noalloc if noalloc else self.L.capib_diagnostics
        st = fn(self.ctx, C.byref(d))
        if st != CAPIB_OK and not (allow_unstable and st == CAPIB_E_UNSTABLE):
            self._check(st)
        return dict(step=d.step, error_flags=d.error_flags, n_bodies=d.n_bodies, mass=d.mass, mom_x=d.mom_x,
                    mom_y=d.mom_y, near_tiles=d.near_tiles, tiles=d.tiles, status=st)

    def sample_members(self, out=None, particle_tag=2, cell_tag=1):
        """Per member: drag, lift, hazard, r, dp, nearest cell, wall shear
        rate, N_L (see capib_sample_members) into a [members][8] float
        tensor on the device (allocated if not given).  Enqueued."""
        if out is None:
            out = self.torch.empty((len(self.bands), 8), dtype=self.torch.float32, device=self.device)
        assert out.dtype == self.torch.float32 and out.is_contiguous() and out.numel() >= 8 * len(self.bands)
        cur = self.torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        self._check(self.L.capib_sample_members(self.ctx, particle_tag, cell_tag, _P(out.data_ptr())))
        # the caller's stream sees the samples only after the library's stream wrote them
        cur.wait_stream(self.stream)
        return out

    def body_diagnostics(self, body):
        d = capib_body_diag()
        self._check(self.L.capib_body_diagnostics(self.ctx, body, C.byref(d)))
        return {k: getattr(d, k) for k, _ in capib_body_diag._fields_ if k != "reserved"}

    def readout(self, cell, particle):
        """(delta_p of the cell, centroid distance r, N_L/N_L0 of the particle)."""
        out = np.zeros(3)
        self._check(self.L.capib_readout(self.ctx, cell, particle, _d(out)))
        return dict(dp=float(out[0]), r=float(out[1]), nl_ratio=float(out[2]))

    def body_state(self, body):
        """x^n, x^n - x^{n-1} and the 9 rigid state values of a body."""
        n = self.nv[body]
        xy, d, r = np.zeros((n, 2)), np.zeros((n, 2)), np.zeros(9)
        self._check(self.L.capib_read_body_state(self.ctx, body, _d(xy), _d(d), _d(r)))
        return dict(xy=xy, dxy_prev=d, rigid=r)

    def save(self):
        n = C.c_size_t()
        self._check(self.L.capib_save(self.ctx, None, C.byref(n)))
        buf = (C.c_char * n.value)()
        self._check(self.L.capib_save(self.ctx, C.cast(buf, _P), C.byref(n)))
        return bytes(buf)

    def load(self, blob):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(self.L.capib_load(self.ctx, C.cast(buf, _P), len(blob)))


def copy_bandwidth(dst, src, stream=None):
    """Enqueues the library's streaming copy of the torch tensor src into dst
    (same byte size, 16-byte aligned) on stream (default: the current one)."""
    import torch
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    st = stream if stream is not None else torch.cuda.current_stream()
    s = load_library().capib_copy_bandwidth(_P(dst.data_ptr()), _P(src.data_ptr()), nbytes, _P(st.cuda_stream))
    if s != CAPIB_OK:
        raise CapibError(s, "capib_copy_bandwidth rejected its arguments")


def fp16_scale_for(cfg, headroom=16.0):
    """Power-of-two scale for FP16 storage of the population deviations.

    Stored deviations from the row reference are bounded by the flow speed
    u (a deviation w_i (3 e.du + drho + ...) with |du|, |drho| <~ u), so the
    scale maps u to 65504 / headroom: the largest normal FP16 value is then
    reached only by deviations `headroom` times the flow speed, and ordinary
    ones keep the full 11-bit significand instead of falling to subnormals."""
    u = float(cfg.meta.get("umax", 0.0))
    if cfg.ux_init is not None:
        u = max(u, float(np.abs(cfg.ux_init).max()))
    if not u > 0.0:
        return 2.0 ** 20
    return 2.0 ** math.floor(math.log2(65504.0 / headroom / u))


def from_ensemble(cfgs, storage=FP32_SHIFTED, fp16_scale=1.0, stream=None, graph=False):
    """Builds one ensemble Simulation from a list of inputs.Config that share
    ny, tau, the drive, walls, the initial profile and the interaction
    constants (member k is cfgs[k]; its bodies are numbered after those of
    the members before it).  Returns the simulation and the first body id of
    each member."""
    c0 = cfgs[0]
    for c in cfgs[1:]:
        same = (c.ny, c.tau, c.gx, c.gy, c.walls, c.rep_pref, c.rep_cut, c.probe_dist) == \
               (c0.ny, c0.tau, c0.gx, c0.gy, c0.walls, c0.rep_pref, c0.rep_cut, c0.probe_dist)
        same = same and ((c.ux_init is None and c0.ux_init is None) or
                         (c.ux_init is not None and c0.ux_init is not None and np.array_equal(c.ux_init, c0.ux_init)))
        if not same:
            raise ValueError("ensemble members must share ny, tau, drive, walls, profile and interactions")
    sim = Simulation(0, c0.ny, c0.tau, c0.gx, c0.gy, c0.walls, storage=storage, fp16_scale=fp16_scale,
                     max_bodies=max(1, sum(len(c.bodies) for c in cfgs)),
                     max_vertices=max(1, sum(c.n_vertices for c in cfgs)),
                     max_sites=max(1, sum(c.n_sites for c in cfgs)), stream=stream, bands=[c.nx for c in cfgs])
    sim.set_interactions(c0.rep_pref, c0.rep_cut, c0.probe_dist)
    sim.init_flow(c0.ux_init)
    first = []
    for k, c in enumerate(cfgs):
        b0 = len(sim.nv)
        first.append(b0)
        for b in c.bodies:
            sim.add_membrane(b.kind, b.xy, b.xy_rest, b.ks, b.kb, b.ka, b.pref, b.rho_r, b.tag, band=k)
        for bd in c.bonds:
            sim.add_bonds(b0 + bd.body, bd.host, bd.frac, bd.sigma, bd.ycr, bd.yeq, bd.kf, bd.kr0, bd.lb, bd.seed)
    if graph:
        sim.set_graph(True)
    return sim, first


def from_config(cfg, storage=FP32_SHIFTED, fp16_scale=1.0, stream=None, graph=False):
    """Builds a Simulation from an inputs.Config (same numbers the oracle gets)."""
    sim = Simulation(cfg.nx, cfg.ny, cfg.tau, cfg.gx, cfg.gy, cfg.walls, storage=storage, fp16_scale=fp16_scale,
                     max_bodies=max(1, len(cfg.bodies)), max_vertices=max(1, cfg.n_vertices),
                     max_sites=max(1, cfg.n_sites), stream=stream)
    sim.set_interactions(cfg.rep_pref, cfg.rep_cut, cfg.probe_dist)
    sim.init_flow(cfg.ux_init)
    for b in cfg.bodies:
        sim.add_membrane(b.kind, b.xy, b.xy_rest, b.ks, b.kb, b.ka, b.pref, b.rho_r, b.tag)
    for bd in cfg.bonds:
        sim.add_bonds(bd.body, bd.host, bd.frac, bd.sigma, bd.ycr, bd.yeq, bd.kf, bd.kr0, bd.lb, bd.seed)
    if graph:
        sim.set_graph(True)
    return sim
