"""Pins of the NumPy surrogate-network oracle: bfloat16 rounding against torch's own
conversion, the back-propagated gradient against central finite differences of the loss
(plain FP64 mode), the FP64 network and its gradient against torch's layers and autograd,
the bfloat16 mode within a first-order bound of its roundings, Adam's first step against its
closed form, the scaler against numpy's moments, and a degenerate network whose output is its
last bias."""
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


def _torch_net(theta):
    """The 4-64-64-2 SiLU network of the parameter vector, built from torch's own layers."""
    p = mlp.unpack(theta)
    net = torch.nn.Sequential(torch.nn.Linear(4, 64), torch.nn.SiLU(), torch.nn.Linear(64, 64), torch.nn.SiLU(),
                              torch.nn.Linear(64, 2)).double()
    with torch.no_grad():
        for layer, (w, b) in zip((net[0], net[2], net[4]), (("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
            layer.weight.copy_(torch.from_numpy(p[w]))
            layer.bias.copy_(torch.from_numpy(p[b]))
    return net


def test_fp64_network_and_gradient_match_torch_autograd():
    """Plain FP64 mode against torch's layers and autograd: output, loss (1/(2B)) sum (y - t)^2
    and the gradient of every weight and bias, including the layout of the parameter vector."""
    rng = np.random.default_rng(7)
    theta = init_params(11).astype(np.float64)
    theta[mlp.N_PARAMS - 66:] += rng.normal(0, 0.2, 66)  # W3 and b3 away from their start
    X = rng.normal(0, 1, (48, 4))
    T = rng.normal(0, 1, (48, 2))
    net = _torch_net(theta)
    y_t = net(torch.from_numpy(X))
    loss_t = 0.5 * ((y_t - torch.from_numpy(T)) ** 2).sum() / X.shape[0]
    loss_t.backward()
    g_t = np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(),
                          net[2].weight.grad.numpy().ravel(), net[2].bias.grad.numpy(),
                          net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy()])
    y_o, _ = mlp.forward(theta, X, bf16=False)
    loss_o, g_o = mlp.loss_and_grad(theta, X, T, bf16=False)
    assert np.allclose(y_o, y_t.detach().numpy(), rtol=1e-12, atol=1e-14)
    assert abs(loss_o - loss_t.item()) <= 1e-12 * loss_t.item()
    assert np.allclose(g_o, g_t, rtol=1e-10, atol=1e-14)


def test_bf16_forward_within_its_rounding_bound():
    """The bfloat16 mode differs from the FP64 network only by its roundings (relative 2^-9
    each): the output error stays within a first-order bound built from the FP64 network's own
    magnitudes, and well above zero (the roundings are really applied)."""
    rng = np.random.default_rng(3)
    theta = init_params(4).astype(np.float64)
    theta[mlp.N_PARAMS - 66:] += rng.normal(0, 0.2, 66)
    X = rng.normal(0, 1, (256, 4))
    y64, c = mlp.forward(theta, X, bf16=False)
    y16, _ = mlp.forward(theta, X, bf16=True)
    p = mlp.unpack(theta)
    u = 2.0 ** -8  # two roundings per product term at 2^-9 each
    a1 = np.abs(X) @ np.abs(p["W1"]).T                        # |x| |W1|
    e1 = u * a1                                                # error of z1
    d1 = np.abs(mlp.dsilu(c["z1"]))
    eh1 = d1 * e1 + 2.0 ** -9 * np.abs(c["h1"])                # error of h1
    a2 = np.abs(c["h1"]) @ np.abs(p["W2"]).T
    e2 = eh1 @ np.abs(p["W2"]).T + u * a2                      # error of z2
    eh2 = np.abs(mlp.dsilu(c["z2"])) * e2 + 2.0 ** -9 * np.abs(c["h2"])
    ey = eh2 @ np.abs(p["W3"]).T + u * (np.abs(c["h2"]) @ np.abs(p["W3"]).T)
    err = np.abs(y16 - y64)
    assert np.all(err <= 1.5 * ey + 1e-12)
    assert err.max() > 1e-4 * np.abs(y64).max()
