"""FP64 reference of the load/hazard surrogate: a multilayer perceptron
with GELU hidden layers, mean-squared-error loss, its gradients by the
chain rule, and the Adam update.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``.  It shares no code with
the HIP kernels.

The network is the one the surrogate direction names: 37 inputs (cell to
particle distance, membrane stretch, aspect ratio, log Ca, cell type, and
a 32-sample wall-shear history), four hidden layers of width 256 with
GELU, three outputs (drag, lift, bond-rupture hazard).

With ``bf16=True`` the arithmetic is FP64 but the values are rounded to
bfloat16 (round to nearest, ties to even, from their FP32 value) at the
points where the GPU stores them in bfloat16: the input, the weights, the
hidden activations, the output gradient and the back-propagated
pre-activation gradients.  With ``bf16=False`` everything is plain FP64,
which is what the finite-difference checks of the gradients use.

Definitions used:
  GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2
  GELU'(z) = Phi(z) + z phi(z),  phi(z) = exp(-z^2 / 2) / sqrt(2 pi)
  loss = mean over the batch and the 3 outputs of (y - t)^2
  Adam (Kingma and Ba, 2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
    p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
"""
import math

import numpy as np

DIMS = [37, 256, 256, 256, 256, 3]
_erf = np.vectorize(math.erf)


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) through FP32; FP64 result."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def init_params(seed=0):
    """Weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases zero: a list of
    (W [out][in], b [out]) in FP64."""
    rng = np.random.default_rng(seed)
    ps = []
    for k_in, k_out in zip(DIMS[:-1], DIMS[1:]):
        a = 1.0 / math.sqrt(k_in)
        ps.append((rng.uniform(-a, a, size=(k_out, k_in)), np.zeros(k_out)))
    return ps


def forward(params, x, bf16_points=True):
    """Returns the output y [n][3] and the cache (inputs of every layer and
    the pre-activations) for the backward pass."""
    r = bf16 if bf16_points else (lambda v: np.asarray(v, dtype=np.float64))
    a = r(x)
    acts, zs = [a], []
    for l, (W, b) in enumerate(params):
        z = a @ r(W).T + b
        if l < len(params) - 1:
            zs.append(z)
            a = r(gelu(z))
            acts.append(a)
        else:
            y = z
    return y, (acts, zs)


def loss_and_grads(params, x, t, bf16_points=True):
    """MSE loss and its gradients [(dW, db)] by the chain rule."""
    r = bf16 if bf16_points else (lambda v: np.asarray(v, dtype=np.float64))
    y, (acts, zs) = forward(params, x, bf16_points)
    n = x.shape[0]
    loss = float(np.mean((y - t) ** 2))
    dz = r(2.0 * (y - t) / (n * t.shape[1]))          # gradient at the output layer
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        grads[l] = (dz.T @ acts[l], dz.sum(axis=0))
        if l > 0:
            da = dz @ r(W)
            dz = r(da * gelu_prime(zs[l - 1]))
    return loss, grads


def adam_step(params, grads, state, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of every parameter array (state: list of (m, v) pairs
    per array, updated in place); t counts updates from 1."""
    out = []
    for k, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            m, v = state[2 * k + j]
            m[...] = b1 * m + (1.0 - b1) * g
            v[...] = b2 * v + (1.0 - b2) * g * g
            mh = m / (1.0 - b1 ** t)
            vh = v / (1.0 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append((new[0], new[1]))
    return out


def adam_state(params):
    st = []
    for W, b in params:
        st.append((np.zeros_like(W), np.zeros_like(W)))
        st.append((np.zeros_like(b), np.zeros_like(b)))
    return st


def flatten(params):
    """FP32 parameter vector in the C-ABI's order: W0, b0, W1, b1, ...,
    each W row-major [out][in]."""
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)


def unflatten(vec):
    ps, o = [], 0
    for k_in, k_out in zip(DIMS[:-1], DIMS[1:]):
        W = np.asarray(vec[o:o + k_in * k_out], dtype=np.float64).reshape(k_out, k_in)
        o += k_in * k_out
        b = np.asarray(vec[o:o + k_out], dtype=np.float64)
        o += k_out
        ps.append((W, b))
    return ps


def n_params():
    return sum(k_in * k_out + k_out for k_in, k_out in zip(DIMS[:-1], DIMS[1:]))
