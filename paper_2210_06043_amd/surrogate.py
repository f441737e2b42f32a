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
    """(X [n][37], T [n][3], member id per row) from a harvest."""
    ns, nm, _ = samples.shape
    X, T, M = [], [], []
    for m, cfg in enumerate(cfgs):
        s = samples[:, m, :]
        ca = cfg.meta["ca"]
        lca = math.log10(ca) if ca > 0 else -6.0
        types = cfg.meta.get("cell_types", [])
        for k in range(HIST - 1, ns):
            cell = int(s[k, 5]) - first[m]
            ctype = float(types[cell]) if 0 <= cell < len(types) else 0.0
            X.append(np.concatenate([[s[k, 3], s[k, 4], cfg.meta["ar"], lca, ctype], s[k - HIST + 1:k + 1, 6]]))
            T.append(s[k, :3])
            M.append(m)
    return np.asarray(X, np.float64), np.asarray(T, np.float64), np.asarray(M)


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
