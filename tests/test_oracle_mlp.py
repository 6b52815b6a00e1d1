"""Pins of the FP64 closure-MLP reference: central finite differences of the
exact FP64 network, the bfloat16 rounding rule, and Adam's closed form."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 36 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3 == 6723


def test_bf16_rounding_rule():
    # exactly representable values pass unchanged
    for v in (1.0, -2.5, 0.15625, 2.0 ** 100, -(2.0 ** -100)):
        assert mlp.bf16(np.float32(v)) == np.float32(v)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1)
    assert mlp.bf16(np.float32(1 + 2 ** -8)) == 1.0
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties go to 1 + 2^-6
    assert mlp.bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6
    # just above the tie rounds up
    assert mlp.bf16(np.float32(1 + 2 ** -8 + 2 ** -20)) == 1 + 2 ** -7
    rng = np.random.default_rng(0)
    x = rng.standard_normal(10000).astype(np.float32)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8 + 1e-45)


def test_gelu_special_values():
    assert mlp.gelu(np.array(0.0)) == 0.0
    assert mlp.gelu(np.array(10.0)) == pytest.approx(10.0, abs=1e-20)
    assert mlp.gelu(np.array(-10.0)) == pytest.approx(0.0, abs=1e-20)
    # gelu(1) = Phi(1) = 0.8413447460685429
    assert mlp.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, rel=1e-14)
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, rtol=1e-8, atol=1e-10)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    w = mlp.init(3)
    w[-3:] = rng.standard_normal(3) * 0.1  # non-zero last layer
    w[-(64 * 3 + 3):-3] = rng.standard_normal(64 * 3) * 0.1
    x = rng.standard_normal((16, 36))
    t = rng.standard_normal((16, 3))
    _, g = mlp.grad(w, x, t, bf16_operands=False)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss(wp, x, t, False) - mlp.loss(wm, x, t, False)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-10), i


def test_zero_last_layer_outputs_zero():
    rng = np.random.default_rng(2)
    y, _ = mlp.forward(mlp.init(1), rng.standard_normal((8, 36)))
    assert np.all(y == 0.0)


def test_adam_first_step_moves_by_lr_times_sign():
    """With bias correction the first Adam step is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w, m, v = mlp.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=1e-3)
    expect = -1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(w, expect, rtol=1e-12, atol=1e-18)


def test_input_noise_generator_is_splitmix64_and_box_muller():
    """The training-input noise: SplitMix64 outputs for the states 0, gamma,
    2 gamma, 3 gamma are the published sequence of seed 0 (Steele, Lea &
    Flood 2014), and the Box-Muller variates are standard normal (moments,
    the two-sided 3-sigma tail, no correlation between steps or features)."""
    gamma = 0x9E3779B97F4A7C15
    states = np.array([(j * gamma) % (1 << 64) for j in range(4)], dtype=np.uint64)
    assert [int(v) for v in mlp.splitmix64_output(states)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    g0 = mlp.input_noise(11, 0, 20000)
    g1 = mlp.input_noise(11, 1, 20000)
    for g in (g0, g1):
        assert g.shape == (20000, 36) and np.isfinite(g).all()
        assert abs(g.mean()) < 0.01 and abs(g.var() - 1.0) < 0.01
        assert abs(np.mean(g ** 3)) < 0.02 and abs(np.mean(g ** 4) - 3.0) < 0.05
        assert 0.0022 < np.mean(np.abs(g) > 3.0) < 0.0032  # 2 (1 - Phi(3)) = 0.0027
    assert abs(np.corrcoef(g0.ravel(), g1.ravel())[0, 1]) < 0.01
    assert abs(np.corrcoef(g0[:, 0], g0[:, 1])[0, 1]) < 0.03
    assert np.array_equal(mlp.input_noise(11, 0, 50), g0[:50])  # counter-based: rows do not depend on the count
