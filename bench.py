"""Throughput of the fused LBM-IB step on one MI355X.

A step is one pass of the whole hot path: interpolation to every vertex and
probe, membrane/interaction/bond/load forces, integration, direct forcing
and spreading, bond kinetics and the lattice sweep.  The default workload is
the paper-scale capillary (3840 x 240 lattice, six cells of 512 vertices, a
discoidal particle of 128 vertices with 200 engaged bonds), inputs resident
in HBM.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LBM-IBM MLUPS & HBM GB/s (FP32 vs FP16-store); batched sweep runs/hour"
HBM_PEAK_GBS = 8000.0


LATTICE_SOURCES = ("capib_dev.hpp", "lattice_dev.hpp", "lattice.hip", "body.hip")
TUBE3D_SOURCES = ("tube3d.hip",)


def kernel_source_hash(sources=LATTICE_SOURCES):
    """Hash of the sources of the lattice launches (their device code and the
    host code that sets their shares of the tiles), comments and blank lines
    left out, so that the counters stay valid across edits of the text."""
    import re
    csrc = os.path.join(ROOT, "paper_2210_06043_amd", "csrc")
    h = hashlib.sha256()
    for f in sources:
        for line in open(os.path.join(csrc, f), encoding="utf-8"):
            code = re.sub(r"//.*", "", line).rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def counters(name, sources=LATTICE_SOURCES):
    """HBM bytes per launch of a lattice kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"{name}_counters.json")
    if not os.path.exists(p):
        return None
    c = json.load(open(p))
    if c.get("source_hash") != kernel_source_hash(sources):
        return None
    return c.get("bytes_per_launch")


def workload(name, seed):
    from paper_2210_06043_amd import inputs
    if name == "c2":
        cfg = inputs.config_c2(seed=seed)
        desc = (f"paper-scale capillary 3840x240 (dx=0.03125um), 6 cells x 512 markers, discoidal particle "
                f"AR={cfg.meta['ar']} Ca={cfg.meta['ca']} x 128 markers, 200 bonds engaged, Re=0.01")
    else:
        cfg = inputs.config_c1(seed=seed)
        desc = "small capillary 480x60, circular cell 256 markers, rigid ellipse 64 markers, 50 bonds, Re=0.01"
    return cfg, desc


def host_cpu():
    """Host core count and CPU model (lscpu, else /proc/cpuinfo)."""
    import subprocess
    model = "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return os.cpu_count(), model


def cpu_baseline(cfg, steps, single_steps):
    """The FP64 oracle on this host's cores: `steps` coupled steps with its
    per-node loops on every core OpenMP is given (the reference state the GPU
    runs are compared against), and `single_steps` on one thread."""
    import oracle
    nproc, model = host_cpu()
    all_threads = oracle.threads()

    def run(n, threads):
        oracle.set_threads(threads)
        s = oracle.Sim(cfg.nx, cfg.ny, cfg.tau, cfg.gx, cfg.gy, cfg.walls)
        s.set_interactions(cfg.rep_pref, cfg.rep_cut, cfg.probe_dist)
        s.init_flow(cfg.ux_init)
        for b in cfg.bodies:
            s.add_body(b.kind, b.xy, b.xy_rest, b.ks, b.kb, b.ka, b.pref, b.rho_r, b.tag)
        for bd in cfg.bonds:
            s.add_bonds(bd.body, bd.host, bd.frac, bd.sigma, bd.ycr, bd.yeq, bd.kf, bd.kr0, bd.lb, bd.seed)
        x0 = [s.vertices(k).copy() for k in range(len(cfg.bodies))]
        t0 = time.perf_counter()
        s.step(n)
        return s, x0, time.perf_counter() - t0

    s1, _, dt1 = run(single_steps, 1)
    del s1
    s, x0, dt = run(steps, all_threads)
    oracle.set_threads(all_threads)
    ref = dict(u=np.stack(s.macro()[1:]), x=[s.vertices(k) for k in range(len(cfg.bodies))], x0=x0,
               n_bound=[s.count_bound(bd.body) for bd in cfg.bonds])
    nodes = cfg.nx * cfg.ny
    out = dict(value=round(nodes * steps / dt / 1e6, 3), unit="MLUPS", cores=all_threads, kind="oracle",
               sample=f"{steps} full coupled steps of the same workload (FP64), OpenMP over the per-node loops on "
                      f"{all_threads} threads, {dt:.1f} s",
               single_thread=dict(value=round(nodes * single_steps / dt1 / 1e6, 3), unit="MLUPS", cores=1,
                                  sample=f"{single_steps} steps on one thread, {dt1:.1f} s"),
               nproc=nproc, cpu_model=model)
    return out, ref


def error_vs_oracle(cfg, storage, scale, steps, ref):
    """Max-norm relative errors of a fresh GPU run of `steps` steps against
    the oracle state: velocity, marker displacement; bond counts."""
    from paper_2210_06043_amd import capib
    g = capib.from_config(cfg, storage=storage, fp16_scale=scale)
    g.step(steps)
    _, ux, uy = g.macro()
    u = np.stack([ux, uy])
    eu = float(np.abs(u - ref["u"]).max() / np.abs(ref["u"]).max())
    ed = 0.0
    for k in range(len(cfg.bodies)):
        d_ref = ref["x"][k] - ref["x0"][k]
        ed = max(ed, float(np.abs(g.vertices(k) - ref["x"][k]).max() / np.abs(d_ref).max()))
    nb = [g.body_diagnostics(bd.body)["n_bound"] for bd in cfg.bonds]
    return dict(velocity_rel=eu, displacement_rel=ed, n_bound_equal=nb == ref["n_bound"], steps=steps)


def measure(cfg, storage, scale, steps, warmup, graph=True):
    """Timed steps and the per-kernel event times.  With graphs, the library
    instantiates every graph when they are enabled (before the warm-up), so
    the timed region only replays them."""
    import torch
    from paper_2210_06043_amd import capib
    sim = capib.from_config(cfg, storage=storage, fp16_scale=scale, graph=graph)
    st = sim.stream
    sim.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    sim.step(steps)
    e1.record(st)
    e1.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    # per-kernel HIP events on the library's stream, same number of steps
    sim.set_timing(True)
    sim.step(steps)
    sim.set_timing(False)
    ph, n, swept = sim.read_timing()
    diag = sim.diagnostics()
    nodes = cfg.nx * cfg.ny
    assert swept.sum() == nodes * n, (swept, nodes, n)   # every node once per step
    # Dominant lattice kernel, 9 reads + 9 writes per node it sweeps (the
    # spread records the near tiles read add well under 1 %), with the nodes
    # each launch swept as the library counted them from each step's
    # near-tile flags.  On a small lattice the membrane launch (k_body_far)
    # sweeps a share of the far tiles and the sweep after it the rest; on a
    # large one the far tiles have a launch beside the membrane phase.
    bytes_per_node = 72 if storage == capib.FP32_SHIFTED else 36
    names = ["k_interp", "k_body_far", "k_lattice_far", "k_lattice_sweep"]
    launch_ms = ph / n
    k = max((1, 2, 3), key=lambda q: launch_ms[q] if swept[q] else -1.0)
    kernel, kernel_ms = names[k], launch_ms[k]
    alg_bytes = bytes_per_node * swept[k] / n
    split = launch_ms[2] > 0
    # "body_far": the membrane launch that also sweeps far tiles
    phases = {"interp": round(launch_ms[0] * 1e3, 3), "body_far" if swept[1] else "body": round(launch_ms[1] * 1e3, 3)}
    if split:
        phases["lattice_far"] = round(launch_ms[2] * 1e3, 3)
    phases["lattice_sweep"] = round(launch_ms[3] * 1e3, 3)
    lattice_ms = sum(launch_ms[q] for q in (1, 2, 3) if swept[q])
    del sim
    torch.cuda.empty_cache()
    return dict(ms=ms, mlups=nodes * steps / (ms * 1e-3) / 1e6, kernel=kernel, kernel_ms=kernel_ms,
                alg_bytes=alg_bytes, achieved=alg_bytes / (kernel_ms * 1e-3) / 1e9, near_tiles=diag["near_tiles"],
                phases=phases, nodes_per_launch={names[q]: int(swept[q] // n) for q in (1, 2, 3) if swept[q]},
                whole_sweep_gbs=bytes_per_node * nodes / (lattice_ms * 1e-3) / 1e9, error_flags=diag["error_flags"])


def _ensemble_step_ms(cfgs, storage, scale, args):
    """ms per step of one ensemble of `cfgs`, and its per-launch timing."""
    import torch
    from paper_2210_06043_amd import capib
    sim, _ = capib.from_ensemble(cfgs, storage=storage, fp16_scale=scale, graph=not args.no_graph)
    sim.step(args.batched_warmup)
    # the library's autotuner picks the launch configuration for this
    # workload (same results for every configuration), outside the timing
    tuned = sim.autotune(steps_per_trial=args.tune_steps) if args.tune_steps else sim.tuning()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(args.batched_steps)
    e1.record(sim.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / args.batched_steps
    sim.set_timing(True)
    sim.step(args.batched_steps)
    sim.set_timing(False)
    ph, n, swept = sim.read_timing()
    diag = sim.diagnostics()
    del sim
    torch.cuda.empty_cache()
    return ms, ph, n, swept, diag, tuned


def _single_step_ms(cfg, storage, scale, args):
    """ms per step of one member run alone as a single lattice."""
    import torch
    from paper_2210_06043_amd import capib
    g = capib.from_config(cfg, storage=storage, fp16_scale=scale, graph=not args.no_graph)
    g.step(200)
    if args.tune_steps:
        g.autotune(steps_per_trial=args.tune_steps)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(g.stream)
    g.step(args.batched_steps)
    b.record(g.stream)
    b.synchronize()
    del g
    return a.elapsed_time(b) / args.batched_steps


def batched(args):
    """The batched ensemble (256 capillaries) against the same members run
    one after another as single lattices, each with the same population
    storage (so at the same accuracy against the oracle): completed
    20k-step runs per hour, from the measured step times.  FP16 storage is
    the configured ensemble; FP32 is reported beside it."""
    from paper_2210_06043_amd import capib, inputs
    cfgs = inputs.config_c3(seed=0, members=args.members)
    scale = capib.fp16_scale_for(cfgs[0])
    nodes = sum(c.nx * c.ny for c in cfgs)
    ms16, ph, n, swept, diag, tune16 = _ensemble_step_ms(cfgs, capib.FP16_SHIFTED, scale, args)
    far_ms = ph[2] / n
    alg = 36 * swept[2] / n   # nodes of the far tiles, counted per step
    ms32, ph32, n32, swept32, diag32, tune32 = _ensemble_step_ms(cfgs, capib.FP32_SHIFTED, 1.0, args)
    far32_ms = ph32[2] / n32
    alg32 = 72 * swept32[2] / n32
    # single-instance step times on an evenly spaced sample of members
    sample = list(range(0, len(cfgs), max(1, len(cfgs) // args.single_sample)))[:args.single_sample]
    t32 = [_single_step_ms(cfgs[k], capib.FP32_SHIFTED, 1.0, args) for k in sample]
    t16 = [_single_step_ms(cfgs[k], capib.FP16_SHIFTED, scale, args) for k in sample]
    steps_per_run = cfgs[0].steps

    def rph(ms, members):
        return members * 3600.0 / (steps_per_run * ms * 1e-3)

    rph16, rph32 = rph(ms16, len(cfgs)), rph(ms32, len(cfgs))
    s16, s32 = rph(float(np.mean(t16)), 1), rph(float(np.mean(t32)), 1)
    return {
        "workload": f"{len(cfgs)} capillaries, lengths U{{256..2048}} x 64, 1-4 cells (128-256 markers), "
                    f"one adhered particle each (64 markers, 20 bonds); one ensemble, FP16 storage",
        "members": len(cfgs), "nodes": nodes, "vertices": sum(c.n_vertices for c in cfgs),
        "steps_per_run": steps_per_run, "ms_per_step": round(ms16, 5),
        "mlups": round(nodes / (ms16 * 1e-3) / 1e6, 1), "runs_per_hour": round(rph16, 1),
        "single_fp16_runs_per_hour": round(s16, 1), "speedup_same_storage": round(rph16 / s16, 2),
        "single_fp32_runs_per_hour": round(s32, 1), "speedup_vs_plain_fp32_single": round(rph16 / s32, 2),
        "fp32_ensemble": {"ms_per_step": round(ms32, 5), "mlups": round(nodes / (ms32 * 1e-3) / 1e6, 1),
                          "runs_per_hour": round(rph32, 1), "speedup_same_storage": round(rph32 / s32, 2),
                          "lattice_far_gbs": round(alg32 / (far32_ms * 1e-3) / 1e9, 1),
                          "tuning": {k: v for k, v in tune32.items() if k != "ms_per_step"},
                          "error_flags": diag32["error_flags"]},
        "tuning": {k: v for k, v in tune16.items() if k != "ms_per_step"},
        "tuning_note": "launch configuration chosen by capib_autotune on each workload "
                       f"({args.tune_steps} steps per trial; singles tuned alike)" if args.tune_steps
                       else "library rules (autotuner off)",
        "equal_accuracy_speedup": {"fp16_ensemble_vs_fp16_single": round(rph16 / s16, 2),
                                   "fp32_ensemble_vs_fp32_single": round(rph32 / s32, 2)},
        "single_sample": f"members {sample}: mean {np.mean(t32) * 1e3:.2f} us/step FP32, "
                         f"{np.mean(t16) * 1e3:.2f} us/step FP16, run one after another",
        "accuracy": "the ensemble and the single runs of each storage take the same arithmetic (FP32: members "
                    "bit-identical to their single runs; FP16: within 1e-3 of the FP64 oracle, tested)",
        "roofline": {"bound": "hbm", "kernel": "k_lattice_far", "achieved": round(alg / (far_ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / (far_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes_per_launch": alg, "avg_launch_us": round(far_ms * 1e3, 3),
                     "traffic": counters("lattice_far_fp16_c3")},
        "phase_us_per_step": {"interp": round(ph[0] / n * 1e3, 3), "body": round(ph[1] / n * 1e3, 3),
                              "lattice_far": round(far_ms * 1e3, 3), "lattice_sweep": round(ph[3] / n * 1e3, 3)},
        "error_flags": diag["error_flags"],
    }


def copy_peak(mib=1024, reps=20):
    """Bandwidth of the library's plain streaming copy (bytes read + written
    per second) on two buffers of `mib` MiB: what a streaming kernel reaches
    on this device, beside the vendor's 8 TB/s."""
    import torch
    from paper_2210_06043_amd import capib
    n = mib << 20
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    for _ in range(3):
        capib.copy_bandwidth(b, a, st)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        capib.copy_bandwidth(b, a, st)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    assert torch.equal(a[:4096], b[:4096])
    del a, b
    torch.cuda.empty_cache()
    return round(2.0 * n / (ms * 1e-3) / 1e9, 1)


def mr_section(args, copy_gbs):
    """The single-lattice HBM case: 16384 x 1024 (16.8 M nodes) with
    paper-scale bodies, FP32 and FP16 storage."""
    from paper_2210_06043_amd import capib, inputs
    cfg = inputs.config_mr()
    scale = capib.fp16_scale_for(cfg)
    out = {"workload": f"single capillary 16384x1024 (dx=0.03125um), 24 cells x 512 markers, discoidal particle "
                       f"AR={cfg.meta['ar']} Ca={cfg.meta['ca']} x 128 markers, 200 bonds, Re=0.01",
           "nodes": cfg.nx * cfg.ny, "vertices": cfg.n_vertices, "steps": args.mr_steps}
    for name, st, sc in (("fp32", capib.FP32_SHIFTED, 1.0), ("fp16", capib.FP16_SHIFTED, scale)):
        m = measure(cfg, st, sc, args.mr_steps, args.mr_warmup, graph=not args.no_graph)
        r = roofline(m, name, "mr")
        r["frac_of_copy_peak"] = round(m["achieved"] / copy_gbs, 4) if copy_gbs else None
        out[name] = {"mlups": round(m["mlups"], 1), "ms_per_step": round(m["ms"] / args.mr_steps, 5),
                     "roofline": r, "phase_us_per_step": m["phases"],
                     "lattice_bandwidth_whole_sweep_gbs": round(m["whole_sweep_gbs"], 1),
                     "error_flags": m["error_flags"]}
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0


def mlp_inference_rate(params, nb=65536, reps=20):
    """Time of one inference batch of the surrogate (65,536 samples) on the
    matrix cores, and its rate in FLOP/s of the unpadded network."""
    import torch
    from paper_2210_06043_amd import mlp, surrogate
    import ctypes
    inf = mlp.Surrogate(nb)
    inf.set_params(params if params is not None else surrogate.init_params(0))
    x = torch.randn((nb, mlp.IN), device=inf.device)
    y = torch.empty((nb, mlp.OUT), dtype=torch.float32, device=inf.device)
    inf.forward(x)
    torch.cuda.synchronize()
    # back-to-back launches on the surrogate's own stream through the C-ABI
    # (input and output resident, no per-call allocation or stream joins)
    xp, yp = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(inf.stream)
    for _ in range(reps):
        inf._check(inf.L.capib_mlp_forward(inf.h, xp, nb, yp))
    e1.record(inf.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    dims = [mlp.IN, mlp.HIDDEN, mlp.HIDDEN, mlp.HIDDEN, mlp.HIDDEN, mlp.OUT]
    flops = 2 * nb * sum(a * b for a, b in zip(dims[:-1], dims[1:]))
    return {"batch": nb, "ms_per_batch": ms, "flops_per_launch": flops, "tflops": flops / (ms * 1e-3) / 1e12,
            "reps": reps}


def surrogate_section(args, batched_out):
    """The load/hazard surrogate screening a parameter sweep: four networks
    trained on the solver's samples of the 256 capillaries of the batched
    workload; the sweep is 32 unseen capillaries with six particle variants
    each, where one solver run per capillary supplies the cell-side features,
    the networks answer the other variants and an uncertain variant falls
    back to the solver (threshold chosen on half of the capillaries for a
    standardised error of 0.1, error and runs measured on the other half).
    Also the inference rate on the matrix cores."""
    from paper_2210_06043_amd import inputs, surrogate
    tr = inputs.config_c3(seed=0, members=args.members)
    res = surrogate.screening_study(tr, sweep_seed=1, cells=32, train_steps=args.train_steps, eps=0.1)
    nets = res.pop("nets")
    rate = mlp_inference_rate(nets[0].get_params())
    nb, ms_inf, flops, tflops = rate["batch"], rate["ms_per_batch"], rate["flops_per_launch"], rate["tflops"]
    out = {
        "workload": f"MLP 37 -> 4 x 256 (GELU) -> 3, BF16 operands / FP32 accumulation (MFMA 32x32x16), "
                    f"4 networks trained on {res['train_samples']} solver samples of {len(tr)} capillaries",
        "train_steps": args.train_steps, "train_batch": 4096, "ms_per_train_step": round(res["ms_per_train_step"], 4),
        "screening": {
            "sweep": "32 unseen capillaries x 6 particle variants (AR 0.3/0.6/0.9, rigid or Ca 1e-4); one solver "
                     "run per capillary supplies the cell-side features; uncertain variants fall back to the solver",
            "stated_error": res["eps"], "uncertainty_threshold": round(res["tau"], 5),
            "evaluation_error_drag_lift_hazard": [round(e, 4) for e in res["eval_error"]],
            "evaluation_solver_runs": res["eval_runs"], "evaluation_answers": res["eval_answers"],
            "fallbacks": res["eval_fallbacks"], "answers_per_solver_run": round(res["answers_per_run"], 3)},
        "inference_batch": nb, "ms_per_inference_batch": round(ms_inf, 4),
        "predictions_per_hour": round(nb / (ms_inf * 1e-3) * 3600.0, 1),
        "roofline": {"bound": "mfma", "kernel": "k_mlp_infer", "achieved": round(tflops, 2),
                     "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None,
                     "algorithmic_flops_per_launch": flops},
    }
    if batched_out:
        # a variant answer costs a solver run of the batched workload without
        # the surrogate, 1 / answers_per_run of one with it (inference time
        # is negligible: one variant's samples take microseconds)
        rph = batched_out["runs_per_hour"]
        out["screening"]["solver_only_answers_per_hour"] = round(rph, 1)
        out["screening"]["screened_answers_per_hour"] = round(rph * res["answers_per_run"], 1)
    return out


def tube3d_section(args):
    """The 3D extension's lattice: D3Q19 BGK with the Guo term in the
    256 x 64 x 64 tube (R = 32) at Re = 0.01, FP32 deviation storage with the
    collision in FP64; back-to-back steps on the library's stream, timed
    with events; the FP64 oracle's error over 20 steps from the same state."""
    import torch
    from paper_2210_06043_amd import inputs, tube3d
    p = inputs.tube3d_params()
    g = tube3d.Tube3D(p["nx"], p["ny"], p["nz"], p["tau"], p["gx"], radius=p["radius"])
    prof = tube3d.hagen_poiseuille(p["ny"], p["nz"], p["radius"], p["tau"], p["gx"])
    g.init_flow(prof)
    g.step(args.tube3d_warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(g.stream)
    g.step(args.tube3d_steps)
    e1.record(g.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / args.tube3d_steps
    n = g.fluid_nodes
    alg = 2 * 19 * 4 * n          # 19 FP32 populations read and written per fluid node
    gbs = alg / (ms * 1e-3) / 1e9
    # the same with FP16 storage (FP32 arithmetic)
    umax = float(prof.max())
    g16 = tube3d.Tube3D(p["nx"], p["ny"], p["nz"], p["tau"], p["gx"], radius=p["radius"],
                        storage=capib_fp16(), fp16_scale=tube3d.fp16_scale_for(umax))
    g16.init_flow(prof)
    g16.step(args.tube3d_warmup)
    torch.cuda.synchronize()
    e0.record(g16.stream)
    g16.step(args.tube3d_steps)
    e1.record(g16.stream)
    e1.synchronize()
    ms16 = e0.elapsed_time(e1) / args.tube3d_steps
    gbs16 = alg / 2 / (ms16 * 1e-3) / 1e9
    fp16 = {"ms_per_step": round(ms16, 5), "mlups": round(n / (ms16 * 1e-3) / 1e6, 1),
            "roofline": {"bound": "hbm", "kernel": "k3_sweep", "achieved": round(gbs16, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs16 / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": alg // 2,
                         "traffic": counters("k3_sweep_fp16_tube", TUBE3D_SOURCES)}}
    # the same FP32 tube with a fixed 2562-vertex sphere of radius 10 on its axis
    # (interpolation + direct forcing per vertex, spread gathered in the sweep)
    xyz, tri = inputs.icosphere(4, 10.0, (0.5 * p["nx"], 0.5 * (p["ny"] - 1) + 0.2, 0.5 * (p["nz"] - 1) - 0.1))
    gb = tube3d.Tube3D(p["nx"], p["ny"], p["nz"], p["tau"], p["gx"], radius=p["radius"], max_vertices=len(xyz))
    gb.init_flow(prof)
    gb.add_fixed_body(xyz, tri)
    gb.step(args.tube3d_warmup)
    torch.cuda.synchronize()
    e0.record(gb.stream)
    gb.step(args.tube3d_steps)
    e1.record(gb.stream)
    e1.synchronize()
    msb = e0.elapsed_time(e1) / args.tube3d_steps
    drag = -gb.body_forces().sum(axis=0)
    body = {"vertices": len(xyz), "triangles": len(tri), "ms_per_step": round(msb, 5),
            "mlups": round(n / (msb * 1e-3) / 1e6, 1), "overhead_us_per_step": round((msb - ms) * 1e3, 2),
            "drag_x_after_warmup_and_steps": float(drag[0]),
            "note": "three launches per step: k3_node_u (velocity of the 7167 stencil nodes, a wave per slot), "
                    "k3_vertex (a wave per vertex), k3_sweep_ib (slots gather their spread force, then the "
                    "ordinary items)"}
    # the same FP32 tube with four 2562-vertex oblate cells and a 642-vertex
    # sphere as deformable membranes (Skalak, area and volume penalties)
    mem = tube3d_membrane_run(p, prof, args.tube3d_warmup, args.tube3d_steps)
    mem["ms_per_step"] = round(mem["ms_per_step"], 5)
    mem["mlups"] = round(n / (mem["ms_per_step"] * 1e-3) / 1e6, 1)
    mem["overhead_us_per_step"] = round((mem["ms_per_step"] - ms) * 1e3, 2)
    # the same with FP16 storage (a timing; parity of FP16 membranes is
    # tested on a smaller tube)
    m16 = tube3d_membrane_run(p, prof, args.tube3d_warmup, args.tube3d_steps, fp16=True)
    mem["fp16_storage"] = {"ms_per_step": round(m16["ms_per_step"], 5),
                           "mlups": round(n / (m16["ms_per_step"] * 1e-3) / 1e6, 1),
                           "bound_after": m16["bound_after"], "error_flags": m16["error_flags"]}
    return {"workload": f"D3Q19 tube {p['nx']}x{p['ny']}x{p['nz']}, radius {p['radius']:g} ({n} fluid nodes), tau 1, "
                        f"Re 0.01 (g = {p['gx']:.4g}), halfway bounce-back walls; FP32 deviation storage, FP64 collision",
            "fluid_nodes": n, "steps": args.tube3d_steps, "ms_per_step": round(ms, 5),
            "mlups": round(n / (ms * 1e-3) / 1e6, 1),
            "roofline": {"bound": "hbm", "kernel": "k3_sweep", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "algorithmic_bytes_per_launch": alg, "traffic": counters("k3_sweep_fp32_tube", TUBE3D_SOURCES),
                         "note": "one launch per step, timed back to back (launch gaps included); the 125 MB "
                                 "working set fits the 256 MB Infinity Cache"},
            "fp16_storage": fp16, "fixed_body": body, "membranes": mem}


def tube3d_membrane_run(p, prof, warmup, steps, fp16=False):
    """The 3D workload (inputs.tube3d_workload): four 2562-vertex oblate
    cells and a 642-vertex oblate particle with 300 ligand sites near the
    wall, in the 256 x 64 x 64 tube; back-to-back steps on the stream; FP32
    deviation storage (FP64 collision), or FP16 (FP32 arithmetic)."""
    import torch
    from paper_2210_06043_amd import inputs, tube3d
    w = inputs.tube3d_workload(p)
    mem = w["cells"] + [w["particle"]]
    kw = dict(storage=capib_fp16(), fp16_scale=tube3d.fp16_scale_for(float(prof.max()))) if fp16 else {}
    g = tube3d.Tube3D(p["nx"], p["ny"], p["nz"], p["tau"], p["gx"], radius=p["radius"], max_membranes=len(mem),
                      max_membrane_vertices=sum(len(m[0]) for m in mem),
                      max_membrane_triangles=sum(len(m[1]) for m in mem), max_sites=len(w["sites"][0]), **kw)
    g.init_flow(prof)
    for (xyz, tri), q in zip(mem, [w["cell"]] * 4 + [w["part"]]):
        g.add_membrane(xyz, tri, **q)
    g.add_bonds(len(mem) - 1, *w["sites"], **w["bonds"])
    g.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(g.stream)
    g.step(steps)
    e1.record(g.stream)
    e1.synchronize()
    t = [g.membrane_totals(m) for m in range(len(mem))]
    return {"membranes": len(mem), "vertices": g.membrane_vertex_count, "triangles": sum(len(m[1]) for m in mem),
            "sites": len(w["sites"][0]), "bound_after": int(g.bonds()[2]),
            "ms_per_step": e0.elapsed_time(e1) / steps, "error_flags": g.error_flags(),
            "volume_drift_max": float(max(abs(x[1] / x[3] - 1) for x in t)),
            "note": "per step: k3_m_first (u* once per node of the work items under the stencils; triangle and edge "
                    "terms, area and volume, the previous step's bond kinetics), k3_m_patch (a workgroup per 32 "
                    "vertices: u* gathered, forces, update, spreading through an LDS box), k3_sweep reading the field "
                    "on flagged items"}


def capib_fp16():
    from paper_2210_06043_amd import capib
    return capib.FP16_SHIFTED


def tube3d_error_vs_oracle(steps=20):
    """Max-norm relative velocity error of the 3D tube against the FP64
    oracle over `steps` steps from the same (GPU-stored) state (part of the
    CPU-baseline leg: the oracle runs on the host)."""
    from oracle import tube3d as otube
    from paper_2210_06043_amd import inputs, tube3d
    p = inputs.tube3d_params()
    g = tube3d.Tube3D(p["nx"], p["ny"], p["nz"], p["tau"], p["gx"], radius=p["radius"])
    g.init_flow(tube3d.hagen_poiseuille(p["ny"], p["nz"], p["radius"], p["tau"], p["gx"]))
    g.step(50)
    o = otube.Tube(p["nx"], p["ny"], p["nz"], p["tau"], p["gx"], radius=p["radius"])
    o.set_populations(g.populations())
    g.step(steps)
    o.step(steps)
    ug, uo = np.stack(g.macro()[1:]), np.stack(o.macro()[1:])
    return float(np.abs(ug - uo).max() / np.abs(uo).max())


def roofline(m, storage_name, workload_name):
    traffic = counters(f"{m['kernel'][2:]}_{storage_name}_{workload_name}")
    return {"bound": "hbm", "kernel": m["kernel"], "achieved": round(m["achieved"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(m["achieved"] / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": int(round(m["alg_bytes"])), "avg_launch_us": round(m["kernel_ms"] * 1e3, 3),
            "near_tiles": m["near_tiles"], "nodes_per_launch": m["nodes_per_launch"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--workload", choices=["c2", "c1"], default="c2")
    # seed 2 draws the rigid (Ca = 0) square particle; the soft draws develop a
    # period-2 wall instability after ~2000 steps
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--storage", choices=["both", "fp32", "fp16"], default="both")
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--cpu-single-steps", type=int, default=30)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="print only the batched-ensemble measurement (for profiling it alone)")
    ap.add_argument("--members", type=int, default=256)
    ap.add_argument("--batched-steps", type=int, default=400)
    ap.add_argument("--batched-warmup", type=int, default=100)
    ap.add_argument("--single-sample", type=int, default=8)
    ap.add_argument("--tune-steps", type=int, default=32,
                    help="steps per autotuner trial for the batched section (0: library rules)")
    ap.add_argument("--no-mr", action="store_true")
    ap.add_argument("--mr-only", action="store_true", help="print only the 16384x1024 measurement")
    ap.add_argument("--mr-steps", type=int, default=200)
    ap.add_argument("--mr-warmup", type=int, default=20)
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-tube3d", action="store_true")
    ap.add_argument("--tube3d-only", action="store_true", help="print only the 3D tube measurement")
    ap.add_argument("--tube3d-steps", type=int, default=1000)
    ap.add_argument("--tube3d-warmup", type=int, default=100)
    ap.add_argument("--harvest-steps", type=int, default=600)
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mlp-only", action="store_true",
                    help="only time the surrogate's inference kernel on random weights (for profiling it alone)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="only run the library's streaming copy of this many MiB (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding across GPUs is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2210_06043_amd import capib

    torch.cuda.set_device(0)
    if args.copy_probe_mb:
        n = args.copy_probe_mb << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            capib.copy_bandwidth(b, a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": n, "copy_bytes_written_per_launch": n}))
        return
    if args.batched_only:
        print(json.dumps({"batched": batched(args)}), flush=True)
        return
    if args.mlp_only:
        print(json.dumps({"mlp_inference": mlp_inference_rate(None)}), flush=True)
        return
    if args.mr_only:
        print(json.dumps({"mr": mr_section(args, None)}), flush=True)
        return
    if args.tube3d_only:
        print(json.dumps({"tube3d": tube3d_section(args)}), flush=True)
        return
    cfg, desc = workload(args.workload, args.seed)
    nodes = cfg.nx * cfg.ny
    scale16 = capib.fp16_scale_for(cfg)
    main_storage = "fp16" if args.storage == "fp16" else "fp32"
    runs = {}
    for name in (["fp32", "fp16"] if args.storage == "both" else [args.storage]):
        st = capib.FP16_SHIFTED if name == "fp16" else capib.FP32_SHIFTED
        runs[name] = measure(cfg, st, scale16 if name == "fp16" else 1.0, args.steps, args.warmup,
                             graph=not args.no_graph)
    m = runs[main_storage]
    copy_gbs = copy_peak()

    out = {
        "metric": METRIC,
        "value": round(m["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms"] / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "nodes": nodes, "population_storage": main_storage + "_deviation",
                   "hip_graphs": not args.no_graph, "vertices": cfg.n_vertices, "sites": cfg.n_sites},
        "roofline": roofline(m, main_storage, args.workload),
        "copy_peak_gbs": copy_gbs,
        "phase_us_per_step": m["phases"],
        "lattice_bandwidth_whole_sweep_gbs": round(m["whole_sweep_gbs"], 1),
        "error_flags": m["error_flags"],
    }
    out["roofline"]["frac_of_copy_peak"] = round(m["achieved"] / copy_gbs, 4)
    if main_storage == "fp32" and "fp16" in runs:
        f = runs["fp16"]
        out["fp16_storage"] = {"value": round(f["mlups"], 1), "unit": "MLUPS",
                               "ms_per_step": round(f["ms"] / args.steps, 5), "fp16_scale": scale16,
                               "roofline": roofline(f, "fp16", args.workload), "phase_us_per_step": f["phases"],
                               "lattice_bandwidth_whole_sweep_gbs": round(f["whole_sweep_gbs"], 1),
                               "error_flags": f["error_flags"]}
    if not args.no_mr:
        out["mr"] = mr_section(args, copy_gbs)
    if not args.no_batched:
        out["batched"] = batched(args)
    if not args.no_tube3d:
        out["tube3d"] = tube3d_section(args)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_section(args, out.get("batched"))
    if not args.no_cpu_baseline:
        base, ref = cpu_baseline(cfg, args.cpu_steps, args.cpu_single_steps)
        out["cpu_baseline"] = base
        out["error_vs_oracle"] = {
            name: error_vs_oracle(cfg, capib.FP16_SHIFTED if name == "fp16" else capib.FP32_SHIFTED,
                                  scale16 if name == "fp16" else 1.0, args.cpu_steps, ref) for name in runs}
        if "tube3d" in out:
            out["tube3d"]["velocity_rel_err_vs_oracle_20_steps"] = tube3d_error_vs_oracle(20)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
