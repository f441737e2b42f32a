"""The surrogate's FP64 reference against what fixes it independently:
the bfloat16 format's definition, closed forms of GELU, central finite
differences of the loss (for every layer's weights and biases), and the
Adam update written out for a single scalar."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_bf16_rounding_definition():
    """Nearest bfloat16 (8 significand bits), ties to even, from FP32."""
    one = 1.0
    ulp = 2.0 ** -7                 # spacing of bfloat16 in [1, 2)
    assert mlp.bf16(one) == one
    assert mlp.bf16(one + 0.25 * ulp) == one                 # below half: down
    assert mlp.bf16(one + 0.75 * ulp) == one + ulp            # above half: up
    assert mlp.bf16(one + 0.5 * ulp) == one                   # tie: to the even significand
    assert mlp.bf16(one + 1.5 * ulp) == one + 2 * ulp         # tie: to the even significand
    assert mlp.bf16(-3.0) == -3.0 and mlp.bf16(0.0) == 0.0
    x = np.random.default_rng(0).standard_normal(1000)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))    # half an ulp: 2^-8 of the binade
    assert np.array_equal(mlp.bf16(r), r)                                   # idempotent


def test_gelu_closed_forms():
    assert mlp.gelu(np.array(0.0)) == 0.0
    # GELU(z) - GELU(-z) = z (Phi(z) + Phi(-z) = 1)
    z = np.linspace(-4, 4, 17)
    np.testing.assert_allclose(mlp.gelu(z) - mlp.gelu(-z), z, rtol=0, atol=1e-15)
    # GELU(1) = Phi(1) = 0.8413447460685429 (standard normal CDF)
    assert abs(mlp.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    # derivative: central differences
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_prime(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), rtol=0, atol=1e-8)
    assert abs(mlp.gelu_prime(np.array(0.0)) - 0.5) < 1e-15


@pytest.fixture(scope="module")
def small():
    """A narrow network of the same structure (widths 6 -> 5 -> 4 -> 2) for
    finite differences, with non-zero biases."""
    rng = np.random.default_rng(3)
    dims = [6, 5, 4, 2]
    ps = [(rng.standard_normal((o, i)) / math.sqrt(i), 0.1 * rng.standard_normal(o))
          for i, o in zip(dims[:-1], dims[1:])]
    x = rng.standard_normal((7, 6))
    t = rng.standard_normal((7, 2))
    return ps, x, t


def test_gradients_match_central_differences(small):
    """Every weight and bias gradient of the chain rule equals the central
    difference of the FP64 loss (no bfloat16 rounding)."""
    ps, x, t = small
    loss, grads = mlp.loss_and_grads(ps, x, t, bf16_points=False)
    h = 1e-6
    for l, (W, b) in enumerate(ps):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            num = np.zeros_like(arr)
            for idx in np.ndindex(arr.shape):
                old = arr[idx]
                arr[idx] = old + h
                lp, _ = mlp.loss_and_grads(ps, x, t, bf16_points=False)
                arr[idx] = old - h
                lm, _ = mlp.loss_and_grads(ps, x, t, bf16_points=False)
                arr[idx] = old
                num[idx] = (lp - lm) / (2 * h)
            np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-9)


def test_linear_network_reduces_to_least_squares_gradient():
    """One linear layer: the gradient is 2/(n m) (X W^T + b - T)^T X."""
    rng = np.random.default_rng(1)
    W, b = rng.standard_normal((3, 4)), rng.standard_normal(3)
    x, t = rng.standard_normal((5, 4)), rng.standard_normal((5, 3))
    loss, g = mlp.loss_and_grads([(W, b)], x, t, bf16_points=False)
    r = x @ W.T + b - t
    assert abs(loss - np.mean(r ** 2)) < 1e-14
    np.testing.assert_allclose(g[0][0], 2.0 / 15.0 * r.T @ x, rtol=1e-13)
    np.testing.assert_allclose(g[0][1], 2.0 / 15.0 * r.sum(0), rtol=1e-13)


def test_adam_first_steps_written_out():
    """First update: m/(1-b1) = g and v/(1-b2) = g^2, so the step is
    -lr g/(|g| + eps); the second follows the recurrences by hand."""
    W = np.array([[0.5]])
    b = np.array([0.0])
    st = mlp.adam_state([(W, b)])
    g1, g2 = 0.3, -0.1
    p1 = mlp.adam_step([(W, b)], [(np.array([[g1]]), np.array([0.0]))], st, lr=0.01, t=1)
    assert abs(p1[0][0][0, 0] - (0.5 - 0.01 * g1 / (abs(g1) + 1e-8))) < 1e-15
    p2 = mlp.adam_step(p1, [(np.array([[g2]]), np.array([0.0]))], st, lr=0.01, t=2)
    m = 0.9 * 0.1 * g1 + 0.1 * g2
    v = 0.999 * 0.001 * g1 * g1 + 0.001 * g2 * g2
    exp = p1[0][0][0, 0] - 0.01 * (m / (1 - 0.81)) / (math.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert abs(p2[0][0][0, 0] - exp) < 1e-15


def test_parameter_vector_layout():
    ps = mlp.init_params(0)
    v = mlp.flatten(ps)
    assert v.size == mlp.n_params() == 37 * 256 + 256 + 3 * (256 * 256 + 256) + 256 * 3 + 3
    back = mlp.unflatten(v)
    for (W, b), (W2, b2) in zip(ps, back):
        np.testing.assert_array_equal(W.astype(np.float32), W2.astype(np.float32))
        np.testing.assert_array_equal(b2, b)
