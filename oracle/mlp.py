"""Plain FP64 reference of the network behind the learned blend coefficient.

TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.

The learned limiter is not in the paper: it is a small multilayer perceptron
that proposes the blend coefficient of a face's cell-average flux (the role
the smoothness indicator of Sec. 3.2 plays), trained on the method's own
theta^s, and always clamped by the density/pressure limiter of Sec. 3.3
exactly as theta^s is, which keeps the admissibility argument of Sec. 3.3
intact.  This module is that network written out in numpy:

  h1 = tanh(W1 x + b1)      W1: 64 x 40
  h2 = tanh(W2 h1 + b2)     W2: 64 x 64
  z  = w3 . h2 + b3         w3: 64
  theta_nn = min(max(z, 0), 1)

Parameters are one flat vector [W1 (row-major, W1[o, i]), b1, W2, b2, w3, b3]
(6849 values).  Training minimises the mean of (z - y)^2 with Adam.  The
inference the stage uses stores the weights W1, W2, w3 and the layer inputs
x, h1 in bfloat16 (round to nearest even) and accumulates in FP32; infer_bf16
takes the same roundings and accumulates in FP64.
"""
from __future__ import annotations

import numpy as np

NIN, NH = 40, 64
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("w3", (NH,)),
         ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(params: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(params[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def forward(params: np.ndarray, X: np.ndarray):
    """z for each row of X (n x 40), and the activations"""
    P = unpack(params)
    h1 = np.tanh(X @ P["W1"].T + P["b1"])
    h2 = np.tanh(h1 @ P["W2"].T + P["b2"])
    z = h2 @ P["w3"] + P["b3"][0]
    return z, (h1, h2)


def loss_and_grad(params: np.ndarray, X: np.ndarray, y: np.ndarray):
    """mean squared error of z against y over the rows of X, and its
    gradient with respect to params (backpropagation)"""
    P = unpack(params)
    n = X.shape[0]
    z, (h1, h2) = forward(params, X)
    r = z - y
    loss = float(np.mean(r * r))
    dz = 2.0 * r / n                              # dL/dz
    g = {"w3": h2.T @ dz, "b3": np.array([dz.sum()])}
    da2 = np.outer(dz, P["w3"]) * (1.0 - h2 * h2)  # dL/d(W2 h1 + b2)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ P["W2"]) * (1.0 - h1 * h1)        # dL/d(W1 x + b1)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return loss, pack(g)


def adam(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """one Adam update (Kingma and Ba), step counted from 1"""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16(x) -> np.ndarray:
    """round to bfloat16 (nearest even), through float32, returned as float64"""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def infer_bf16(params: np.ndarray, X: np.ndarray) -> np.ndarray:
    """theta_nn for each row of X with the stage's storage precisions:
    W1, W2, w3 and the layer inputs x, h1 rounded to bfloat16, biases and
    h2 in FP32 (here FP64), sums in FP64; clamped to [0, 1]"""
    P = unpack(params)
    W1, W2, w3 = bf16(P["W1"]), bf16(P["W2"]), bf16(P["w3"])
    b1, b2, b3 = (np.asarray(P[k], dtype=np.float32).astype(np.float64) for k in ("b1", "b2", "b3"))
    h1 = np.tanh(bf16(X) @ W1.T + b1)
    h2 = np.tanh(bf16(h1) @ W2.T + b2)
    z = h2 @ w3 + b3[0]
    return np.clip(z, 0.0, 1.0)
