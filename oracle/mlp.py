"""FP64 NumPy oracle of the surrogate network (test infrastructure only).

Network: 4 -> 64 -> 64 -> 2 with SiLU hidden activations, trained on the mean squared error
L = (1/(2B)) sum_{rows, outputs} (y - t)^2 with Adam (Kingma & Ba: beta1 0.9, beta2 0.999,
eps 1e-8, bias-corrected moments).  Inputs and targets are standardized with their
population mean and standard deviation over the training set.

With ``bf16=True`` the values are rounded to bfloat16 (round to nearest, ties to even) at the
points where the GPU kernels hold them in bfloat16: the standardized inputs, the three weight
matrices used in the products, both hidden activations after SiLU, and the hidden-2 gradient
fed to the 64x64 products.  All arithmetic is otherwise FP64 (the GPU accumulates in FP32).
With ``bf16=False`` it is a plain FP64 network, used to pin the gradient by finite
differences.

Parameter vector layout: W1 (64 x 4, row-major), b1 (64), W2 (64 x 64, W2[n][k] maps hidden-1
unit k to hidden-2 unit n), b2 (64), W3 (2 x 64), b3 (2) -- 4,610 numbers.
"""
import numpy as np

N_IN, N_H, N_OUT = 4, 64, 2
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_OUT, N_H)),
         ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out = {}
    o = 0
    for name, shp in SIZES:
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k], np.float64).reshape(shp)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SIZES])


def to_bf16(x):
    """Round to the nearest bfloat16 (ties to even) through the float32 bit pattern."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def fit_scaler(X, Y):
    """Population mean and standard deviation of every input and target column."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    xs = X.std(axis=0)
    ys = Y.std(axis=0)
    xs[xs == 0] = 1.0
    ys[ys == 0] = 1.0
    return {"x_mu": X.mean(axis=0), "x_sd": xs, "y_mu": Y.mean(axis=0), "y_sd": ys}


def _round(x, bf16):
    return to_bf16(x) if bf16 else np.asarray(x, np.float64)


def forward(theta, Xs, bf16=True):
    """Forward pass on standardized inputs; returns the output and the cached values."""
    p = unpack(theta)
    x = _round(Xs, bf16)
    W1, W2, W3 = _round(p["W1"], bf16), _round(p["W2"], bf16), _round(p["W3"], bf16)
    z1 = x @ W1.T + p["b1"]
    h1 = _round(silu(z1), bf16)
    z2 = h1 @ W2.T + p["b2"]
    h2 = _round(silu(z2), bf16)
    y = h2 @ W3.T + p["b3"]
    return y, {"x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "W1": W1, "W2": W2, "W3": W3}


def loss_and_grad(theta, Xs, Ts, bf16=True):
    """Loss (1/(2B)) sum (y - t)^2 and its gradient with respect to the FP32 master weights
    (through the rounded copies, as straight-through: d/dW of round(W) is taken as 1)."""
    B = Xs.shape[0]
    y, c = forward(theta, Xs, bf16)
    d = y - Ts
    loss = 0.5 * np.sum(d * d) / B
    dy = d / B
    gW3 = dy.T @ c["h2"]
    gb3 = dy.sum(axis=0)
    dz2 = (dy @ c["W3"]) * dsilu(c["z2"])
    dz2r = _round(dz2, bf16)
    gW2 = dz2r.T @ c["h1"]
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2r @ c["W2"]) * dsilu(c["z1"])
    gW1 = dz1.T @ c["x"]
    gb1 = dz1.sum(axis=0)
    return loss, pack({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3})


def standardize(X, Y, sc):
    Xs = (np.asarray(X, np.float64) - sc["x_mu"]) / sc["x_sd"]
    Ts = None if Y is None else (np.asarray(Y, np.float64) - sc["y_mu"]) / sc["y_sd"]
    return Xs, Ts


def adam(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1**t)
    vh = v / (1.0 - beta2**t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta, X, Y, rows, batch, steps, lr, sc, bf16=True):
    """Minibatch k uses rows[k*batch:(k+1)*batch].  Returns (theta, per-step losses)."""
    theta = np.asarray(theta, np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = []
    Xs, Ts = standardize(X, Y, sc)
    for k in range(steps):
        idx = rows[k * batch:(k + 1) * batch]
        loss, g = loss_and_grad(theta, Xs[idx], Ts[idx], bf16)
        theta, m, v = adam(theta, m, v, g, k + 1, lr)
        losses.append(loss)
    return theta, np.array(losses)


def infer(theta, X, sc, bf16=True):
    Xs, _ = standardize(X, None, sc)
    y, _ = forward(theta, Xs, bf16)
    return y * sc["y_sd"] + sc["y_mu"]
