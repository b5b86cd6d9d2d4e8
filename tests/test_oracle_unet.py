"""Pins of the FP64 warm-start network oracle (no GPU)."""
import numpy as np
import pytest
from scipy import signal

from oracle import unet as U


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -2.5, 3.0e38, 1e-40])
    y = U.bf16(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1.0) wins
    assert y[0] == 1.0 and y[1] == 1.0
    assert y[2] == 1.0 + 2 ** -6  # tie rounds to the even neighbour
    assert y[3] == 1.0 + 2 ** -7 and y[4] == -2.5
    assert np.isfinite(y[5])


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 6, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = U.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate2d(x[n, :, :, c], w[o, :, :, c], mode="same")
                             for c in range(3))
            assert np.allclose(y[n, :, :, o], ref, atol=1e-12)


def test_pool_and_transposed_conv_by_definition():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 4, 6, 2))
    y, idx = U.maxpool2(x)
    for i in range(2):
        for j in range(3):
            for c in range(2):
                win = x[0, 2 * i:2 * i + 2, 2 * j:2 * j + 2, c].ravel()
                assert y[0, i, j, c] == win.max() and idx[0, i, j, c] == int(np.argmax(win))
    w = rng.standard_normal((2, 2, 2, 3))
    b = rng.standard_normal(3)
    t = U.convT2(x, w, b)
    for i in range(4):
        for j in range(6):
            for a in range(2):
                for e in range(2):
                    assert np.allclose(t[0, 2 * i + a, 2 * j + e], b + x[0, i, j] @ w[a, e])


@pytest.mark.parametrize("cout", [1, 3])
def test_gradients_by_finite_differences(cout):
    rng = np.random.default_rng(2)
    base, levels = 3, 4
    p = U.init_params(rng, base, levels, cout)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((2, 8, 8, 1))
    t = rng.standard_normal((2, 8, 8, cout))
    y, cache = U.forward(p, x, levels)
    assert y.shape == t.shape
    loss, gy = U.mse(y, t)
    g = U.backward(cache, gy, levels)
    assert set(g) == set(p)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for i in rng.choice(flat.size, min(3, flat.size), replace=False):
            old = flat[i]
            flat[i] = old + eps
            lp, _ = U.mse(U.forward(p, x, levels)[0], t)
            flat[i] = old - eps
            lm, _ = U.mse(U.forward(p, x, levels)[0], t)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            assert g[k].reshape(-1)[i] == pytest.approx(fd, rel=1e-4, abs=1e-8), k


def test_parameter_count_of_the_32_channel_network():
    n = sum(int(np.prod(s)) for _, s in U.param_shapes(32, 4))
    assert 1.9e6 < n < 2.0e6
    # three outputs add two rows of the 1x1 head
    n3 = sum(int(np.prod(s)) for _, s in U.param_shapes(32, 4, cout=3))
    assert n3 - n == 2 * (32 + 1)


def test_adam_on_a_quadratic():
    """Adam with a fixed step: the first update moves every coordinate by lr
    (bias-corrected m/sqrt(v) = sign(g)), and it converges on a quadratic."""
    p = {"w": np.array([3.0, -2.0])}
    m = {"w": np.zeros(2)}
    v = {"w": np.zeros(2)}
    U.adam_step(p, {"w": 2 * p["w"]}, m, v, 1, 0.1)
    assert np.allclose(p["w"], [2.9, -1.9], atol=1e-7)
    for t in range(2, 2000):
        U.adam_step(p, {"w": 2 * p["w"]}, m, v, t, 0.05)
    assert np.all(np.abs(p["w"]) < 1e-2)
