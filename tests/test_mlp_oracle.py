"""Pins of the network oracle (CPU): finite differences, the logistic-regression
special case, a closed-form Adam step, bfloat16 rounding against torch."""
import math

import numpy as np
import pytest

import synth
from oracle import mlp


def _data(seed, B=16):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, 64))
    y = (rng.random(B) < 0.5).astype(np.float64)
    return x, y


def test_parameter_count():
    assert mlp.N_PARAMS == 82689
    assert synth.mlp_init_params(0).size == mlp.N_PARAMS


def test_gradient_matches_central_differences():
    d = mlp.unpack(synth.mlp_init_params(3).astype(np.float64) * 0.5)
    x, y = _data(1)
    _, g = mlp.loss_and_grad(d, x, y)
    p = mlp.pack(d)
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False), [mlp.N_PARAMS - 1]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        zp, _ = mlp.forward(mlp.unpack(pp), x)
        zm, _ = mlp.forward(mlp.unpack(pm), x)
        fd = (mlp.bce_loss(zp, y) - mlp.bce_loss(zm, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10


def test_reduces_to_logistic_regression():
    rng = np.random.default_rng(4)
    B = 32
    x = np.abs(rng.standard_normal((B, 64)))          # non-negative: ReLU is the identity
    y = (rng.random(B) < 0.5).astype(np.float64)
    d = {"W1": np.vstack([np.eye(64), np.zeros((192, 64))]), "b1": np.zeros(256),
         "W2": np.eye(256), "b2": np.zeros(256), "w3": np.zeros(256), "b3": np.array([0.3])}
    wl = rng.standard_normal(64) * 0.2
    d["w3"][:64] = wl
    z, _ = mlp.forward(d, x)
    assert np.allclose(z, x @ wl + 0.3)
    loss, g = mlp.loss_and_grad(d, x, y)
    s = 1 / (1 + np.exp(-(x @ wl + 0.3)))
    gw = mlp.unpack(g)
    assert np.allclose(gw["w3"][:64], x.T @ (s - y) / B, rtol=1e-12, atol=1e-15)
    assert np.allclose(gw["b3"][0], np.mean(s - y), rtol=1e-12)
    assert loss == pytest.approx(np.mean(-y * np.log(s) - (1 - y) * np.log(1 - s)), rel=1e-12)


def test_bce_at_zero_logit_is_log2():
    assert mlp.bce_loss(np.zeros(5), np.array([0, 1, 0, 1, 1.0])) == pytest.approx(math.log(2))


def test_first_adam_step_is_a_sign_step():
    rng = np.random.default_rng(5)
    p, g = rng.standard_normal(100), rng.standard_normal(100)
    p1, m, v = mlp.adam(p, np.zeros(100), np.zeros(100), g, 1, 1e-3, eps=0.0)
    assert np.allclose(p1, p - 1e-3 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.standard_normal(4000).astype(np.float32) * 10.0 ** rng.integers(-8, 8, 4000),
                        np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)
