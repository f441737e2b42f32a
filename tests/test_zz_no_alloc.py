"""capib_diagnostics_noalloc, the diagnostics entry point for callers that
cannot allocate device memory: its FP64 partial sums live in a fixed array
of the library instead of the workspace.  Through the C-ABI it returns what
capib_diagnostics returns (the same kernels summing in the same order), on
two calls in a row, the second on a smaller lattice than the first, and it
refuses a lattice whose partials do not fit the array.  (Collected last:
the suite runs with -x, so a failure here hides no other test.)"""
import ctypes as C

import pytest

from helpers import gpu_sim, say
from paper_2210_06043_amd import capib, inputs


def test_noalloc_refuses_lattices_beyond_its_scratch():
    """Host-side check, no GPU needed: 512 x 400 tiles of 64 x 4 nodes need
    more partials than the fixed array holds."""
    L = capib.load_library()
    lat = capib.capib_lattice(512 * 64, 400 * 4, 1.0, 0.0, 0.0, 3, capib.FP32_SHIFTED, 1.0, 1, 1, 1)
    ctx = C.c_void_p()
    assert L.capib_create(C.byref(lat), None, C.byref(ctx)) == capib.CAPIB_OK
    try:
        d = capib.capib_diag()
        assert L.capib_diagnostics_noalloc(ctx, C.byref(d)) == capib.CAPIB_E_CAPACITY
        msg = L.capib_last_error(ctx).decode()
        assert "scratch" in msg and "tiles" in msg, msg
    finally:
        L.capib_destroy(ctx)


@pytest.mark.gpu
def test_noalloc_diagnostics_equal_the_workspace_path():
    results = []
    for cfg, steps in ((inputs.config_c1(), 40), (inputs.config_tiny(), 25)):
        g = gpu_sim(cfg, graph=True)
        g.step(steps)
        a = g.diagnostics()
        b = g.diagnostics(noalloc=True)
        say(f"{cfg.name}: workspace {a}; no-alloc {b}")
        for key in ("step", "error_flags", "n_bodies", "near_tiles", "tiles", "status"):
            assert a[key] == b[key], key
        # the same partials summed in the same fixed order: identical FP64 totals
        for key in ("mass", "mom_x", "mom_y"):
            assert a[key] == b[key], key
        results.append(b)
    assert results[1]["tiles"] < results[0]["tiles"]
