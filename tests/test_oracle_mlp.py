"""Pins of the NumPy surrogate-network oracle: bfloat16 rounding against torch's own
conversion, the back-propagated gradient against central finite differences of the loss
(plain FP64 mode), Adam's first step against its closed form, the scaler against numpy's
moments, and a degenerate network whose output is its last bias."""
import numpy as np
import pytest
import torch

from oracle import mlp
from workloads.surrogate import init_params, toy_dataset, row_order


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 10000), rng.normal(0, 1e-30, 100), rng.normal(0, 1e30, 100),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38]]).astype(np.float32)
    ours = mlp.to_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_gradient_matches_finite_differences():
    theta = init_params(3).astype(np.float64)
    rng = np.random.default_rng(1)
    theta[mlp.N_PARAMS - 2:] = rng.normal(0, 0.1, 2)
    X = rng.normal(0, 1, (32, 4))
    T = rng.normal(0, 1, (32, 2))
    _, g = mlp.loss_and_grad(theta, X, T, bf16=False)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss_and_grad(tp, X, T, bf16=False)[0] - mlp.loss_and_grad(tm, X, T, bf16=False)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-10)


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so the update is
    -lr g / (|g| + eps), i.e. lr times the sign of the gradient for |g| >> eps."""
    theta = np.zeros(5)
    g = np.array([2.0, -3.0, 1e-3, -5e-4, 0.0])
    t1, m, v = mlp.adam(theta, np.zeros(5), np.zeros(5), g, 1, 0.01)
    assert np.allclose(t1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_scaler_moments():
    X, Y = toy_dataset(500, 2)
    sc = mlp.fit_scaler(X, Y)
    assert np.allclose(sc["x_mu"], X.astype(np.float64).mean(axis=0))
    assert np.allclose(sc["y_sd"], Y.astype(np.float64).std(axis=0))


def test_zero_hidden_weights_give_last_bias():
    theta = np.zeros(mlp.N_PARAMS)
    theta[-2:] = [0.25, -1.5]
    y, _ = mlp.forward(theta, np.random.default_rng(0).normal(0, 1, (7, 4)))
    assert np.array_equal(y, np.tile([0.25, -1.5], (7, 1)))


def test_oracle_training_reduces_loss():
    X, Y = toy_dataset(1024, 4)
    sc = mlp.fit_scaler(X, Y)
    rows = row_order(1024, 64, 300, 5)
    _, losses = mlp.train(init_params(5), X, Y, rows, 64, 300, 3e-3, sc)
    assert losses[-20:].mean() < 0.1 * losses[:5].mean()
