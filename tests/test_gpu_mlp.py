"""GPU parity of the surrogate network kernels (BF16 MFMA, FP32 accumulation) against the
NumPy oracle that rounds to bfloat16 at the same points and accumulates in FP64.

Tolerances (fixed before measuring):
  gradient: normwise relative difference <= 1e-3 per parameter block.  The two sides differ
    by FP32-vs-FP64 accumulation (~1e-7 relative) and, through that, by occasional
    bfloat16 rounding flips of hidden activations (one bf16 ulp = 2^-8 on about one element
    in 10^4), which move a block's gradient by ~2^-8 / sqrt(B) ~ 2.5e-4;
  inference: standardized outputs within 2e-2 absolute everywhere and 1e-4 on 99 % of rows;
  training 50 Adam steps: master weights within 1e-3 normwise relative, losses within 1e-3.
"""
import numpy as np
import pytest

from oracle import mlp
from workloads.surrogate import init_params, row_order, toy_dataset

from _helpers import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

BLOCKS = [(0, 256), (256, 320), (320, 4416), (4416, 4480), (4480, 4608), (4608, 4610)]


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda") if dtype is None else t.to(device="cuda", dtype=dtype)


def _oracle_scaler(sc):
    return {k: np.asarray(v, np.float64) for k, v in sc.items()}


@pytest.mark.parametrize("batch", [32, 128, 256])
def test_gradient_matches_oracle(batch):
    import paper_1307_3711_amd as lc
    X, Y = toy_dataset(1000, 7)
    theta = init_params(7)
    net = lc.Surrogate(theta)
    Xd, Yd = _dev(X), _dev(Y)
    net.fit_scaler(Xd, Yd)
    _, sc_gpu = net.params()
    sc = mlp.fit_scaler(X, Y)
    for k in sc:
        assert np.allclose(sc_gpu[k], sc[k], rtol=1e-6)
    rows = row_order(1000, batch, 1, 8)
    g, loss = net.grad(Xd, Yd, _dev(rows), batch)
    g = g.cpu().numpy().astype(np.float64)
    Xs, Ts = mlp.standardize(X, Y, _oracle_scaler(sc_gpu))
    lo, go = mlp.loss_and_grad(theta.astype(np.float64), Xs[rows], Ts[rows], bf16=True)
    assert float(loss.cpu()[0]) == pytest.approx(lo, rel=1e-4)
    for a, b in BLOCKS:
        err = np.linalg.norm(g[a:b] - go[a:b]) / np.linalg.norm(go[a:b])
        print(f"batch {batch} block {a}:{b} rel err {err:.2e}", flush=True)
        assert err <= 1e-3


def test_inference_matches_oracle_ragged():
    import paper_1307_3711_amd as lc
    X, Y = toy_dataset(4099, 9)
    theta = init_params(9)
    net = lc.Surrogate(theta)
    Xd = _dev(X)
    net.fit_scaler(Xd, _dev(Y))
    _, sc = net.params()
    out = net.infer(Xd).cpu().numpy().astype(np.float64)
    ref = mlp.infer(theta.astype(np.float64), X, _oracle_scaler(sc), bf16=True)
    d = np.abs(out - ref) / sc["y_sd"]
    print(f"inference max |d| {d.max():.2e}, 99th pct {np.quantile(d, 0.99):.2e}", flush=True)
    assert d.max() <= 2e-2 and np.quantile(d, 0.99) <= 1e-4
    assert net.infer(_dev(X[:0])).shape == (0, 2)


def test_training_matches_oracle_and_is_reproducible():
    import paper_1307_3711_amd as lc
    X, Y = toy_dataset(2048, 10)
    theta = init_params(10)
    steps, batch, lr = 50, 128, 2e-3
    rows = row_order(2048, batch, steps, 11)
    outs = []
    for _ in range(2):
        net = lc.Surrogate(theta)
        Xd, Yd = _dev(X), _dev(Y)
        net.fit_scaler(Xd, Yd)
        losses = net.train(Xd, Yd, _dev(rows), batch, steps, lr).cpu().numpy()
        outs.append((net.params(), losses))
    (p1, sc1), l1 = outs[0]
    (p2, _), l2 = outs[1]
    assert np.array_equal(p1, p2) and np.array_equal(l1, l2)
    po, lo = mlp.train(theta.astype(np.float64), X, Y, rows, batch, steps, lr, _oracle_scaler(sc1), bf16=True)
    err = np.linalg.norm(p1 - po) / np.linalg.norm(po)
    print(f"train 50 steps: weights rel err {err:.2e}; loss rel err {np.max(np.abs(l1 - lo) / lo):.2e}", flush=True)
    assert err <= 1e-3
    assert np.max(np.abs(l1 - lo) / lo) <= 1e-3


def test_training_learns_toy_function():
    import paper_1307_3711_amd as lc
    X, Y = toy_dataset(4096, 12)
    net = lc.Surrogate(init_params(12))
    Xd, Yd = _dev(X), _dev(Y)
    net.fit_scaler(Xd, Yd)
    losses = net.train(Xd, Yd, _dev(row_order(4096, 256, 2000, 13)), 256, 2000, 3e-3).cpu().numpy()
    assert losses[-50:].mean() < 0.02 * losses[:5].mean()


def test_training_rejects_bad_rows():
    import paper_1307_3711_amd as lc
    X, Y = toy_dataset(100, 1)
    net = lc.Surrogate(init_params(1))
    rows = np.full(64, 5000, np.int32)
    with pytest.raises(lc.LcError):
        net.train(_dev(X), _dev(Y), _dev(rows), 64, 1, 1e-3)
    with pytest.raises(lc.LcError):
        net.train(_dev(X), _dev(Y), _dev(rows), 48, 1, 1e-3)
