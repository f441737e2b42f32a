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
