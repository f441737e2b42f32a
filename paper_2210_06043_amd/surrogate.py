"""The load/hazard surrogate's data and training loop.

Data comes from the solver: an ensemble of capillaries is advanced on the
GPU and, every `every` steps, capib_sample_members records per member the
particle's drag, lift and bond-rupture hazard with the nearest cell's
distance and stretch and the wall shear rate (all in a device buffer; one
copy to the host at the end).  A sample of member m at time s pairs the
features

    r, dp, aspect ratio, log10 Ca (1e-6 for the rigid class), cell type
    (1 biconcave, 0 globular), and the wall shear rate at the last 32
    sampling times

with the targets (drag, lift, hazard) at s.  Features and targets are
standardised with the training set's mean and spread.  Training and
inference run in the surrogate's HIP kernels (capib_mlp); this module only
arranges arrays."""
import math
import time

import numpy as np

from . import capib, mlp

HIST = 32
PARTICLE, CELL = 2, 1


def harvest(cfgs, steps, every=2, storage=capib.FP16_SHIFTED, graph=True):
    """Runs the members of `cfgs` as one ensemble for `steps` steps and
    samples them every `every` steps.  Returns an array [samples][members][8]
    (capib_sample_members order) and the ensemble's step time in ms."""
    import torch
    scale = capib.fp16_scale_for(cfgs[0]) if storage == capib.FP16_SHIFTED else 1.0
    sim, first = capib.from_ensemble(cfgs, storage=storage, fp16_scale=scale, graph=graph)
    ns = steps // every
    buf = torch.zeros((ns, len(cfgs), 8), dtype=torch.float32, device=sim.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(ns):
        sim.step(every)
        sim.sample_members(buf[k])
    sim.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / (ns * every)
    d = sim.diagnostics()
    if d["error_flags"]:
        raise RuntimeError(f"ensemble went unstable (flags {d['error_flags']})")
    return buf.cpu().numpy(), ms, first


def features(samples, cfgs, first):
    """(X [n][37], T [n][3], member id per row) from a harvest: for member m
    and sampling time k >= HIST - 1, the row (r, dp, aspect ratio, log10 Ca,
    cell type, wall shear at times k - HIST + 1 .. k) with targets (drag,
    lift, hazard) at k."""
    ns, nm, _ = samples.shape
    nk = ns - HIST + 1
    if nk <= 0:
        return np.zeros((0, 5 + HIST)), np.zeros((0, 3)), np.zeros(0, dtype=np.int64)
    S = np.asarray(samples, np.float64)
    X = np.empty((nm, nk, 5 + HIST))
    for m, cfg in enumerate(cfgs):
        s = S[:, m, :]
        ca = cfg.meta["ca"]
        types = np.asarray(cfg.meta.get("cell_types", []), np.float64)
        cell = s[HIST - 1:, 5].astype(np.int64) - first[m]
        ok = (cell >= 0) & (cell < len(types))
        X[m, :, 0] = s[HIST - 1:, 3]
        X[m, :, 1] = s[HIST - 1:, 4]
        X[m, :, 2] = cfg.meta["ar"]
        X[m, :, 3] = math.log10(ca) if ca > 0 else -6.0
        X[m, :, 4] = np.where(ok, types[np.where(ok, cell, 0)] if len(types) else 0.0, 0.0)
        X[m, :, 5:] = np.lib.stride_tricks.sliding_window_view(s[:, 6], HIST)
    T = np.transpose(S[HIST - 1:, :, :3], (1, 0, 2)).reshape(nm * nk, 3)
    M = np.repeat(np.arange(nm), nk)
    return X.reshape(nm * nk, 5 + HIST), T, M


class Standardiser:
    def __init__(self, A):
        self.mu = A.mean(0)
        self.sd = A.std(0)
        self.sd[self.sd == 0] = 1.0

    def __call__(self, A):
        return ((A - self.mu) / self.sd).astype(np.float32)

    def back(self, A):
        return A * self.sd + self.mu


def init_params(seed=0):
    """Weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases zero, in the
    C-ABI's parameter order."""
    rng = np.random.default_rng(seed)
    dims = [mlp.IN, mlp.HIDDEN, mlp.HIDDEN, mlp.HIDDEN, mlp.HIDDEN, mlp.OUT]
    parts = []
    for k_in, k_out in zip(dims[:-1], dims[1:]):
        a = 1.0 / math.sqrt(k_in)
        parts += [rng.uniform(-a, a, size=k_out * k_in), np.zeros(k_out)]
    return np.concatenate(parts).astype(np.float32)


def train(Xs, Ts, steps, batch=4096, lr=1e-3, seed=0, lr_final=1e-5):
    """Adam on minibatches drawn with replacement from the standardised
    training set, learning rate decayed geometrically to lr_final.  Returns
    the surrogate and the mean time per training step (ms)."""
    import torch
    s = mlp.Surrogate(batch)
    s.set_params(init_params(seed))
    dev = s.device
    X = torch.as_tensor(Xs, device=dev)
    T = torch.as_tensor(Ts, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    decay = (lr_final / lr) ** (1.0 / max(1, steps - 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        idx = torch.randint(0, X.shape[0], (batch,), device=dev, generator=g)
        xb, tb = X[idx].contiguous(), T[idx].contiguous()
        s.train_step(xb, tb, lr * decay ** k)
    s.synchronize()
    return s, (time.perf_counter() - t0) * 1e3 / steps


def predict(s, Xs):
    """Batched inference (chunks of the surrogate's batch size)."""
    import torch
    out = []
    for a in range(0, Xs.shape[0], s.max_batch):
        out.append(s.forward(torch.as_tensor(Xs[a:a + s.max_batch], device=s.device)))
    s.synchronize()
    return torch.cat(out).cpu().numpy()


# ---- uncertainty and screening ---------------------------------------------------------

def train_ensemble(Xs, Ts, k=4, steps=1000, batch=4096, seed=0):
    """k networks trained alike from different initial weights and
    minibatch streams (seeds seed .. seed + k - 1); their spread is the
    surrogate's own estimate of its uncertainty."""
    nets, ms = [], []
    for j in range(k):
        net, m = train(Xs, Ts, steps=steps, batch=batch, seed=seed + j)
        nets.append(net)
        ms.append(m)
    return nets, float(np.mean(ms))


def predict_ensemble(nets, Xs):
    """Mean and standard deviation over the networks (standardised units)."""
    P = np.stack([predict(n, Xs) for n in nets])
    return P.mean(0), P.std(0)


# Particle variants of the screened sweep: aspect ratio x Ca (0 = rigid),
# and the variant whose solver run supplies the cell-side features
VARIANTS = [(ar, ca) for ar in (0.3, 0.6, 0.9) for ca in (0.0, 1e-4)]
REFERENCE = (0.6, 1e-4)


def sweep_configs(seed, cells):
    """The sweep: for each of `cells` capillaries drawn from stream `seed`
    (cells, lengths and placement as in the batched workload), the particle
    variants of VARIANTS (same capillary, same bond draws)."""
    from . import inputs
    return [[inputs.c3_member(seed, c, ar=ar, ca=ca) for (ar, ca) in VARIANTS] for c in range(cells)]


def screen(nets, fx, ft, sweep, S, first, tau, rows):
    """Answers of the screened sweep for the capillaries `rows`.

    S is the solver's harvest of the whole sweep as one ensemble (member
    c * len(VARIANTS) + v is variant v of capillary c): the targets the
    screened answers are judged against.  For each capillary the reference
    variant's run is the one solver run made; every other variant is
    predicted by the networks from the reference run's cell-side features
    (r, dp, cell type, wall shear history) with its own aspect ratio and
    Ca.  A variant whose predicted uncertainty (the networks' spread,
    largest over the three outputs, averaged over the run's samples)
    exceeds tau falls back to the solver: its answer is the solver's, at the
    cost of one more run.  Returns (answers, truth, fallback count, solver
    runs made, variant answers given)."""
    nv = len(VARIANTS)
    ref = VARIANTS.index(REFERENCE)
    answers, truth = [], []
    runs = fallbacks = given = 0
    for c in rows:
        row = sweep[c]
        mr = c * nv + ref
        Xr, _, _ = features(S[:, mr:mr + 1, :], [row[ref]], [first[mr]])
        runs += 1
        for v, cfg in enumerate(row):
            m = c * nv + v
            _, Tv, _ = features(S[:, m:m + 1, :], [cfg], [first[m]])
            truth.append(Tv)
            given += 1
            if v == ref:
                answers.append(Tv)
                continue
            Xv = Xr.copy()
            Xv[:, 2] = cfg.meta["ar"]
            Xv[:, 3] = math.log10(cfg.meta["ca"]) if cfg.meta["ca"] > 0 else -6.0
            mu, sd = predict_ensemble(nets, fx(Xv))
            if float(sd.max(axis=1).mean()) > tau:
                fallbacks += 1
                runs += 1
                answers.append(Tv)
            else:
                answers.append(ft.back(mu))
    return answers, truth, fallbacks, runs, given


def screened_error(answers, truth, ft):
    """Standardised mean squared error of the answers over every sample."""
    A = np.concatenate(answers)
    T = np.concatenate(truth)
    return np.mean(((A - T) / ft.sd) ** 2, axis=0)


def screening_study(train_cfgs, sweep_seed=1, cells=32, steps=600, every=2, nets=4, train_steps=1000,
                    eps=0.1):
    """The screened sweep against the solver alone, at a stated accuracy.

    Trains `nets` networks on the solver's harvest of `train_cfgs`; harvests
    the sweep (cells capillaries of stream sweep_seed, every particle
    variant); picks on the first half of the capillaries (calibration) the
    largest uncertainty threshold whose screened answers stay within eps
    (standardised mean squared error, every output), and reports on the
    other half (evaluation) the error reached, the solver runs made and
    the variant answers given per solver run."""
    S, ms_h, first = harvest(train_cfgs, steps, every=every)
    X, T, _ = features(S, train_cfgs, first)
    fx, ft = Standardiser(X), Standardiser(T)
    ens, ms_train = train_ensemble(fx(X), ft(T), k=nets, steps=train_steps)
    sweep = sweep_configs(sweep_seed, cells)
    flat = [cfg for row in sweep for cfg in row]
    S2, _, first2 = harvest(flat, steps, every=every)
    cal, ev = list(range(cells // 2)), list(range(cells // 2, cells))
    # candidate thresholds: none, every spread seen on the calibration set, all
    taus = [0.0]
    for c in cal:
        mr = c * len(VARIANTS) + VARIANTS.index(REFERENCE)
        Xr, _, _ = features(S2[:, mr:mr + 1, :], [sweep[c][VARIANTS.index(REFERENCE)]], [first2[mr]])
        for ar, ca in VARIANTS:
            Xv = Xr.copy()
            Xv[:, 2] = ar
            Xv[:, 3] = math.log10(ca) if ca > 0 else -6.0
            taus.append(float(predict_ensemble(ens, fx(Xv))[1].max(axis=1).mean()))
    taus = sorted(set(taus)) + [float("inf")]
    best = 0.0
    table = []
    for tau in taus:
        a, t, fb, runs, given = screen(ens, fx, ft, sweep, S2, first2, tau, cal)
        err = screened_error(a, t, ft)
        table.append((tau, float(err.max()), runs, given))
        if err.max() <= eps:
            best = tau
    a, t, fb, runs, given = screen(ens, fx, ft, sweep, S2, first2, best, ev)
    err = screened_error(a, t, ft)
    # without screening every variant is a solver run
    return dict(eps=eps, tau=best, eval_error=[float(e) for e in err], eval_runs=runs, eval_answers=given,
                eval_fallbacks=fb, answers_per_run=given / runs, calibration=table, ms_per_train_step=ms_train,
                train_samples=int(X.shape[0]), sweep_members=len(flat), harvest_ms_per_step=ms_h, nets=ens)


def paper_scale_study(train_members=256, test_members=32, train_steps_solver=7876, test_steps_solver=2062, every=2,
                      train_steps=1000, seed=11):
    """The surrogate trained on samples harvested from paper-scale runs.

    Training: train_members paper-scale channels (3840 x 240, six cells,
    the particle's aspect ratio and Ca drawn as in the paper-scale draw, the
    row of cells shifted by U(-150, 150) nodes; inputs.config_c2_placed) run
    as one FP16 ensemble for train_steps_solver steps and sampled every
    `every` steps: 256 x 3,907 = 1.0e6 samples at the defaults.  Held out:
    test_members channels of another stream.  Returns the held-out
    standardised mean squared error per output against the mean guess, the
    sample counts and the timings."""
    from . import inputs
    tr = [inputs.config_c2_placed(seed, k) for k in range(train_members)]
    te = [inputs.config_c2_placed(seed + 1, k) for k in range(test_members)]
    S, ms, first = harvest(tr, train_steps_solver, every=every)
    X, T, _ = features(S, tr, first)
    del S
    S2, ms2, first2 = harvest(te, test_steps_solver, every=every)
    X2, T2, _ = features(S2, te, first2)
    fx, ft = Standardiser(X), Standardiser(T)
    net, ms_train = train(fx(X), ft(T), steps=train_steps, batch=4096)
    P = predict(net, fx(X2))
    err = np.mean((P - ft(T2)) ** 2, axis=0)
    base = np.mean(ft(T2) ** 2, axis=0)
    return dict(train_samples=int(X.shape[0]), test_samples=int(X2.shape[0]), err=[float(e) for e in err],
                mean_guess=[float(b) for b in base], harvest_ms_per_step=ms, ms_per_train_step=ms_train,
                finite=bool(np.all(np.isfinite(P))))
