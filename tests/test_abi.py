"""The C-ABI library builds, loads and exports every symbol its header
declares; host-side argument validation works without a GPU (no compute
calls are made here)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2210_06043_amd import capib, mlp, tube3d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "capib.h")
MLP_HEADER = os.path.join(ROOT, "include", "capib_mlp.h")
HEADER3D = os.path.join(ROOT, "include", "capib3d.h")


def declared_functions(header=HEADER, prefix="capib_"):
    src = open(header).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["capib_create", "capib_bind_workspace", "capib_init_flow", "capib_add_membrane",
                 "capib_add_bonds", "capib_step", "capib_read_macro", "capib_read_vertices", "capib_read_bonds",
                 "capib_diagnostics", "capib_save", "capib_load", "capib_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L = capib.load_library()
    names = declared_functions() + declared_functions(MLP_HEADER) + declared_functions(HEADER3D, "capib3d_")
    for name in names:
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", capib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (capib3?d?_\w+)", out))
    assert set(names) <= exported


def test_binding_covers_the_header():
    assert set(capib.SIGNATURES) == set(declared_functions())
    assert set(mlp.SIGNATURES) == set(declared_functions(MLP_HEADER))
    assert set(tube3d.SIGNATURES) == set(declared_functions(HEADER3D, "capib3d_"))


def test_tube3d_create_validates_without_a_gpu():
    """capib3d_create checks the lattice on the host and sizes the workspace
    (two FP32 population buffers of 19 planes with a 64-aligned pitch, the
    column tables, the FP64 read-out and the partial sums)."""
    L = tube3d._lib()
    ctx = C.c_void_p()
    bad = [tube3d.capib3d_lattice(0, 8, 8, 1.0, 0.0, tube3d.TUBE, 3.0, 0, 1.0),
           tube3d.capib3d_lattice(8, 8, 8, 0.5, 0.0, tube3d.TUBE, 3.0, 0, 1.0),
           tube3d.capib3d_lattice(8, 8, 8, 1.0, 0.0, tube3d.TUBE, 0.0, 0, 1.0),
           tube3d.capib3d_lattice(8, 8, 8, 1.0, 0.0, 7, 3.0, 0, 1.0),
           tube3d.capib3d_lattice(8, 8, 8, 1.0, 0.0, tube3d.TUBE, 3.0, 5, 1.0),
           tube3d.capib3d_lattice(8, 8, 8, 1.0, 0.0, tube3d.TUBE, 3.0, capib.FP16_SHIFTED, 3.0),
           tube3d.capib3d_lattice(8, 8, 8, 1.0, 0.0, tube3d.TUBE, 3.0, 0, 1.0, -1),
           tube3d.capib3d_lattice(8, 8, 8, 1.0, 0.0, tube3d.TUBE, 3.0, 0, 1.0, 0, 1, 0, 0),
           tube3d.capib3d_lattice(8, 8, 8, 1.0, 0.0, tube3d.TUBE, 3.0, 0, 1.0, 0, 1, 162, 0)]
    for lat in bad:
        assert L.capib3d_create(C.byref(lat), None, C.byref(ctx)) == capib.CAPIB_E_ARG
    lat = tube3d.capib3d_lattice(256, 64, 64, 1.0, 1e-7, tube3d.TUBE, 32.0, 0, 1.0)
    assert L.capib3d_create(C.byref(lat), None, C.byref(ctx)) == capib.CAPIB_OK
    try:
        n = L.capib3d_fluid_nodes(ctx)
        assert n == 256 * 3228   # fluid columns of a 64 x 64 cross-section with R = 32
        assert L.capib3d_workspace_bytes(ctx) >= 2 * 19 * 256 * 64 * 64 * 4
        assert L.capib3d_step(ctx, 1) == capib.CAPIB_E_STATE   # no workspace bound
        X = np.zeros(3)
        assert L.capib3d_add_fixed_body(ctx, 1, X.ctypes.data_as(C.POINTER(C.c_double)), 0, None,
                                        None) == capib.CAPIB_E_STATE
        assert L.capib3d_vertices(ctx) == 0
    finally:
        L.capib3d_destroy(ctx)
    # room for fixed-body vertices: stencil nodes, weights, places and contributions of every lane
    lat = tube3d.capib3d_lattice(256, 64, 64, 1.0, 1e-7, tube3d.TUBE, 32.0, 0, 1.0, 2562)
    assert L.capib3d_create(C.byref(lat), None, C.byref(ctx)) == capib.CAPIB_OK
    try:
        assert L.capib3d_workspace_bytes(ctx) >= 2 * 19 * 256 * 64 * 64 * 4 + 2562 * 64 * (4 + 8 + 4 + 24)
    finally:
        L.capib3d_destroy(ctx)


def test_surrogate_parameter_count_matches_the_oracle():
    from oracle import mlp as omlp
    src = open(MLP_HEADER).read()
    n = int(re.search(r"CAPIB_MLP_PARAMS = (\d+)", src).group(1))
    assert n == mlp.N_PARAMS == omlp.n_params()


def test_surrogate_create_validates_without_a_gpu():
    L = mlp._lib()
    h = C.c_void_p()
    assert L.capib_mlp_create(0, None, C.byref(h)) == capib.CAPIB_E_ARG
    assert L.capib_mlp_create(1000, None, C.byref(h)) == capib.CAPIB_OK
    n = L.capib_mlp_workspace_bytes(h)
    assert n % 256 == 0 and n > 4 * 4 * mlp.N_PARAMS        # master weights, gradients, Adam moments
    x = C.c_void_p(256)
    assert L.capib_mlp_forward(h, x, 10, x) == capib.CAPIB_E_STATE    # no workspace bound
    L.capib_mlp_destroy(h)


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and field offsets of the ABI structs seen by a C compiler equal
    the ctypes mirrors of the binding."""
    structs = {
        "capib_lattice": capib.capib_lattice, "capib_membrane": capib.capib_membrane,
        "capib_bonds": capib.capib_bonds, "capib_diag": capib.capib_diag,
        "capib_body_diag": capib.capib_body_diag,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for sname, cls in structs.items():
        lines.append(f'printf("{sname} %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{sname}.{fname} %zu\\n", offsetof({sname}, {fname}));')
    lines.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", str(c), "-o", str(exe)])
    got = dict(ln.split() for ln in subprocess.check_output([str(exe)], text=True).splitlines())
    for sname, cls in structs.items():
        assert int(got[sname]) == C.sizeof(cls), sname
        for fname, _ in cls._fields_:
            assert int(got[f"{sname}.{fname}"]) == getattr(cls, fname).offset, f"{sname}.{fname}"


def _create(**kw):
    L = capib.load_library()
    base = dict(nx=32, ny=16, tau=1.0, gx=0.0, gy=0.0, walls=3, storage=0, fp16_scale=1.0, max_bodies=2,
                max_vertices=64, max_sites=16)
    base.update(kw)
    lat = capib.capib_lattice(**base)
    ctx = C.c_void_p()
    st = L.capib_create(C.byref(lat), None, C.byref(ctx))
    return L, st, ctx


@pytest.mark.parametrize("bad", [dict(tau=0.5), dict(tau=0.3), dict(walls=1), dict(ny=1), dict(nx=0),
                                 dict(storage=7), dict(storage=1, fp16_scale=3.0), dict(tau=float("nan")),
                                 dict(max_sites=-1)])
def test_create_rejects_bad_lattices(bad):
    L, st, ctx = _create(**bad)
    assert st == capib.CAPIB_E_ARG
    assert not ctx.value


def test_create_sizes_the_workspace_and_checks_order():
    L, st, ctx = _create()
    assert st == capib.CAPIB_OK
    n = L.capib_workspace_bytes(ctx)
    # two population buffers of 9 x 16 x 64 floats at least
    assert n >= 2 * 9 * 16 * 64 * 4 and n % 256 == 0
    # nothing may run before a workspace is bound
    assert L.capib_step(ctx, 1) == capib.CAPIB_E_STATE
    assert b"workspace" in L.capib_last_error(ctx)
    assert L.capib_bind_workspace(ctx, C.c_void_p(12345), n) == capib.CAPIB_E_ARG   # misaligned
    L.capib_destroy(ctx)
    L2, st2, ctx2 = _create(storage=1, fp16_scale=2.0 ** 16)
    assert st2 == capib.CAPIB_OK
    assert L2.capib_workspace_bytes(ctx2) < n      # FP16 populations take half the bytes
    L2.capib_destroy(ctx2)


def _create_ensemble(widths, **kw):
    L = capib.load_library()
    base = dict(nx=0, ny=16, tau=1.0, gx=0.0, gy=0.0, walls=3, storage=0, fp16_scale=1.0, max_bodies=2,
                max_vertices=64, max_sites=16)
    base.update(kw)
    lat = capib.capib_lattice(**base)
    ctx = C.c_void_p()
    w = (C.c_int32 * max(1, len(widths)))(*widths)
    st = L.capib_create_ensemble(C.byref(lat), len(widths), w, None, C.byref(ctx))
    return L, st, ctx


@pytest.mark.parametrize("widths,kw", [([], {}), ([32, 0], {}), ([32, 64], dict(ny=18)),
                                        ([32, 64], dict(tau=0.5))])
def test_create_ensemble_rejects_bad_members(widths, kw):
    """No members, a zero width, members whose rows are not whole tile rows,
    or a bad shared lattice parameter are refused."""
    L, st, ctx = _create_ensemble(widths, **kw)
    assert st == capib.CAPIB_E_ARG
    assert not ctx.value


def test_create_ensemble_sizes_the_stack():
    """An ensemble of members of widths 32, 200 and 64 is sized as a stack of
    three 16-row bands of the widest member; one band equals a lattice."""
    L, st, ctx = _create_ensemble([32, 200, 64])
    assert st == capib.CAPIB_OK
    n3 = L.capib_workspace_bytes(ctx)
    assert n3 >= 2 * 9 * (3 * 16) * 256 * 4
    L.capib_destroy(ctx)
    L1, st1, ctx1 = _create_ensemble([200])
    L2, st2, ctx2 = _create(nx=200)
    assert st1 == st2 == capib.CAPIB_OK
    assert L1.capib_workspace_bytes(ctx1) == L2.capib_workspace_bytes(ctx2)
    L1.capib_destroy(ctx1)
    L2.capib_destroy(ctx2)
