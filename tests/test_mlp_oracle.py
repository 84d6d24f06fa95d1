"""Pins of the FP64 network oracle (CPU): finite-difference gradients, closed
forms of the loss and of Adam's first step, BF16 rounding cases."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2603_15186_amd.synth import mlp_init


def _data(seed, n=40):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 8))
    y = (rng.uniform(size=n) < 0.4).astype(np.float64)
    return X, y


def test_layout_and_init():
    assert M.N_PARAMS == 1377
    p = mlp_init(3)
    assert p.dtype == np.float32 and p.size == 1377
    q = M.unpack(p)
    assert q["W1"].shape == (32, 8) and q["W2"].shape == (32, 32) and q["w3"].shape == (32,)
    assert np.all(q["b1"] == 0) and q["b3"] == 0
    assert np.abs(q["W1"]).max() <= np.sqrt(6 / 8) and np.abs(q["W2"]).max() <= np.sqrt(6 / 32)
    np.testing.assert_array_equal(M.pack(q), p.astype(np.float64))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    p = mlp_init(seed).astype(np.float64)
    rng = np.random.default_rng(seed)
    p[M.N_PARAMS - 1] = 0.3
    p[256:288] = rng.normal(0, 0.3, 32)          # nonzero biases
    X, y = _data(seed)
    g = M.grad(p, X, y)
    h = 1e-6
    for k in rng.choice(M.N_PARAMS, 120, replace=False):
        e = np.zeros_like(p); e[k] = h
        fd = (M.loss(p + e, X, y) - M.loss(p - e, X, y)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g).max()) + 1e-9, (k, fd, g[k])


def test_loss_closed_form_for_a_constant_network():
    """All weights zero, b3 = c: z = c for every sample, so the loss is
    log(1 + e^c) - mean(y) c and d loss / d b3 = sigmoid(c) - mean(y)."""
    p = np.zeros(M.N_PARAMS)
    c = 0.7
    p[-1] = c
    X, y = _data(5, 17)
    assert M.loss(p, X, y) == pytest.approx(np.log1p(np.exp(c)) - y.mean() * c, rel=1e-14)
    g = M.grad(p, X, y)
    assert g[-1] == pytest.approx(1 / (1 + np.exp(-c)) - y.mean(), rel=1e-14)
    assert np.all(g[:-1] == 0)


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so the step is
    lr g / (|g| + eps)."""
    g = np.array([0.5, -2e-3, 0.0, 3.0])
    p = np.array([1.0, 2.0, 3.0, 4.0])
    p1, m, v = M.adam(p, np.zeros(4), np.zeros(4), g, 1, 0.01)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_bf16_rounding_is_nearest_even():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)               # BF16 spacing in [1, 2)
    cases = {
        1.0: 1.0,
        float(one + ulp / 2): 1.0,            # tie: to even (1.0)
        float(one + ulp + ulp / 2): float(one + 2 * ulp),   # tie: to even (1 + 2 ulp)
        float(one + ulp / 2 + np.float32(2.0 ** -20)): float(one + ulp),
        -3.140625: -3.140625,
    }
    for x, want in cases.items():
        assert M.bf16_value(M.bf16_bits(np.float32(x))) == want, x
