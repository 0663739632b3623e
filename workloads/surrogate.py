"""Seeded inputs of the surrogate network: initial weights and minibatch row orders.

Initial weights are uniform in +-1/sqrt(fan_in) (the usual default for dense layers), drawn
from numpy's Philox keyed by (seed, 11); biases start at zero.  Row orders are epoch-wise
permutations of the training rows drawn from Philox keyed by (seed, 12).  Nothing here
evaluates the network.
"""
import numpy as np

N_IN, N_H, N_OUT = 4, 64, 2


def init_params(seed):
    rng = np.random.Generator(np.random.Philox(key=[int(seed), 11]))
    parts = []
    for fan_out, fan_in in [(N_H, N_IN), (N_H, N_H), (N_OUT, N_H)]:
        a = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-a, a, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def row_order(n_rows, batch, steps, seed):
    """steps*batch row indices: concatenated random permutations of range(n_rows)."""
    rng = np.random.Generator(np.random.Philox(key=[int(seed), 12]))
    need = steps * batch
    out = []
    while sum(len(o) for o in out) < need:
        out.append(rng.permutation(n_rows))
    return np.concatenate(out)[:need].astype(np.int32)


def toy_dataset(n, seed):
    """A smooth synthetic regression set for tests of the training machinery: four features
    in the ranges of the surrogate's standardized-before log inputs, two targets that are
    fixed smooth functions of them."""
    rng = np.random.Generator(np.random.Philox(key=[int(seed), 13]))
    X = np.stack([rng.uniform(np.log(2.0), np.log(10.0), n), rng.uniform(5.0, 12.0, n),
                  rng.uniform(np.log(1e15), np.log(1e17), n), rng.uniform(np.log(20.0), np.log(100.0), n)],
                 axis=1)
    y0 = 0.8 * X[:, 0] + 0.3 * np.sin(X[:, 1]) + 0.5 * (X[:, 2] - 36.0) - 0.2 * X[:, 3]
    y1 = 1.0 + 2.0 * np.tanh(0.5 * (X[:, 2] - 36.5)) + 0.1 * X[:, 1]
    return X.astype(np.float32), np.stack([y0, y1], axis=1).astype(np.float32)
