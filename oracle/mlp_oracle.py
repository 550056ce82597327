"""FP64 CPU oracle of the learned-bandwidth network (test infrastructure only).

A 4-layer perceptron 32 -> 128 -> 128 -> 128 -> 16 (24 features and 3 outputs,
zero padded), ReLU between layers, trained by mean squared error. The GPU
kernels keep FP32 master parameters, multiply BF16 operands (weights,
activations and, in the backward pass, the output gradients) and accumulate in
FP32. The oracle computes the same network in FP64 and takes the same
precision decisions: ``rnd`` is applied wherever the kernels round an operand
to BF16. With ``rnd`` the identity it is the plain FP64 network, which the
pins check against finite differences.

Layer l (1-based): z_l = a_{l-1} W_l + b_l with W_l stored k-major (in x out),
a_l = relu(z_l) for l < 4, y = z_4. Loss = mean over rows of sum_k (y_k - t_k)^2
(padded output columns have zero targets and zero weights).
"""
from __future__ import annotations

import numpy as np

N_IN, N_IN_PAD, N_HID, N_OUT, N_OUT_PAD = 24, 32, 128, 3, 16
SHAPES = [(N_IN_PAD, N_HID), (N_HID, N_HID), (N_HID, N_HID), (N_HID, N_OUT_PAD)]


def param_count() -> int:
    return sum(k * n + n for k, n in SHAPES)


def unpack(theta):
    """Flat FP32/FP64 parameter vector -> [(W_l, b_l)] in the kernels' order: W1, b1, ..., W4, b4."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for k, n in SHAPES:
        W = theta[o:o + k * n].reshape(k, n)
        o += k * n
        b = theta[o:o + n]
        o += n
        out.append((W, b))
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def bf16(x) -> np.ndarray:
    """Round FP64 values to the nearest BF16 (ties to even), returned as FP64.

    Goes through FP32 first, as the kernels hold FP32 values when they round."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def ident(x):
    return np.asarray(x, dtype=np.float64)


def forward(theta, X, rnd=bf16):
    """Returns y (rows x 16) and the layer inputs a_0..a_3 as the matmuls see them."""
    L = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a = np.zeros((X.shape[0], N_IN_PAD))
    a[:, :X.shape[1]] = X
    a = rnd(a)
    acts = [a]
    for i, (W, b) in enumerate(L):
        z = a @ rnd(W) + b
        if i == 3:
            return z, acts
        a = rnd(np.maximum(z, 0.0))
        acts.append(a)


def loss_and_grad(theta, X, T, rnd=bf16):
    """Mean squared error over the rows and its gradient w.r.t. the flat parameters."""
    L = unpack(theta)
    y, acts = forward(theta, X, rnd)
    B = y.shape[0]
    Tp = np.zeros_like(y)
    Tp[:, :N_OUT] = T
    r = y - Tp
    loss = float(np.sum(r * r) / B)
    dz = 2.0 * r / B
    grads = [None] * 4
    for i in (3, 2, 1, 0):
        W, _ = L[i]
        dzr = rnd(dz)
        grads[i] = (acts[i].T @ dzr, dz.sum(axis=0))
        if i > 0:
            da = dzr @ rnd(W).T
            dz = da * (acts[i] > 0)
    return loss, pack(grads)


def adam(theta, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (bias-corrected moments); returns the new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
