"""Shared test helpers: build the oracle and the HIP simulation from one config."""
import numpy as np

import oracle
from paper_2210_06043_amd import inputs


def oracle_sim(cfg: inputs.Config) -> "oracle.Sim":
    s = oracle.Sim(cfg.nx, cfg.ny, cfg.tau, cfg.gx, cfg.gy, cfg.walls)
    s.set_interactions(cfg.rep_pref, cfg.rep_cut, cfg.probe_dist)
    s.init_flow(cfg.ux_init)
    for b in cfg.bodies:
        s.add_body(b.kind, b.xy, b.xy_rest, b.ks, b.kb, b.ka, b.pref, b.rho_r, b.tag)
    for bd in cfg.bonds:
        s.add_bonds(bd.body, bd.host, bd.frac, bd.sigma, bd.ycr, bd.yeq, bd.kf, bd.kr0, bd.lb, bd.seed)
    return s


def gpu_sim(cfg: inputs.Config, **kw):
    from paper_2210_06043_amd import capib
    return capib.from_config(cfg, **kw)


def rel_max(a, b):
    """max |a - b| / max |b| (max-norm relative error)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def say(*a):
    print(*a, flush=True)


def oracle_steps(o, steps, label="oracle", chunk=250):
    """Advances the oracle, printing progress every `chunk` steps of a long run."""
    import time
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        o.step(n)
        done += n
        if steps > chunk:
            say(f"{label}: oracle step {done}/{steps} ({time.perf_counter() - t0:.0f} s)")


def check_bonds(o, g, cfg, label, first=0, require_flips=False):
    """Bond states, anchors and N_L of the GPU run equal the oracle's.

    Both codes draw the same numbers (the counter-based generator keyed by
    seed, step and site), so they take the same decisions unless the
    oracle's draw fell closer to its probability, or a site's gap closer to
    y_cr, than the GPU's values of P and of the gap can differ from the
    oracle's.  Those differences are bounded from the measured position
    error e of the bonded bodies: the Bell probability moves by at most
    P e / l_B plus FP32 rounding (relative 1e-5 is generous), the gap by e;
    with a factor 10 of safety both must clear the oracle's smallest margins
    (relative |draw - P| / P, and |gap - y_cr|).  A configuration that does
    not clear them fails here: it is re-seeded, not skipped.  Returns the
    number of bond state changes the oracle took."""
    if not cfg.bonds:
        return 0
    err = 0.0
    for bd in cfg.bonds:
        err = max(err, float(np.abs(g.vertices(first + bd.body) - o.vertices(bd.body)).max()))
    lb = min(bd.lb for bd in cfg.bonds)
    thr_p = 1e-5 + 10.0 * err / lb
    thr_g = 10.0 * err + 1e-9
    mp, mg = o.margins()
    say(f"{label}: bonded-body position error {err:.2e}; decision margins |r-P|/P {mp:.2e} (bound {thr_p:.2e}), "
        f"|gap-ycr| {mg:.2e} (bound {thr_g:.2e}); {o.flips} bond flips")
    assert mp > thr_p and mg > thr_g, f"{label}: a bond decision lies within the error bound; re-seed the bonds"
    if require_flips:
        assert o.flips > 0, f"{label}: no bond changed state, the comparison would be trivial"
    for bd in cfg.bonds:
        so, ao = o.bonds(bd.body)
        sg, ag = g.bonds(first + bd.body)
        assert np.array_equal(so, sg), label
        np.testing.assert_allclose(ag[so == 1], ao[so == 1], rtol=0, atol=10.0 * err + 1e-7)
        assert g.body_diagnostics(first + bd.body)["n_bound"] == o.count_bound(bd.body) == int(so.sum())
    return o.flips


def load_gpu_state_into(o, g, cfg):
    """Restarts the oracle `o` (built from cfg) from the state of the
    single-lattice GPU run `g`, promoted to FP64: populations, step index,
    per body x^n, the BDF2 histories and the rigid state, bond states and
    anchors."""
    o.set_populations(g.read_populations())
    o.set_step(g.diagnostics()["step"])
    for k in range(len(cfg.bodies)):
        st = g.body_state(k)
        o.set_body_state(k, st["xy"], st["dxy_prev"], st["rigid"])
    for bd in cfg.bonds:
        o.set_bonds(bd.body, *g.bonds(bd.body))
    o.reset_margins()
