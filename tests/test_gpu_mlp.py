"""The learned-bandwidth network's kernels (MFMA BF16 products, FP32
accumulation) against the FP64 network oracle that rounds the same operands
to BF16.

Bars: every output and every gradient entry within 2^-9 (half a BF16 unit in
the last place) of the largest magnitude of its block (the outputs, or one
weight or bias block): the kernels accumulate in FP32 and may round an
activation to the neighbouring BF16 value where the FP64 value sits next to a
rounding boundary, which moves a downstream product term by at most one BF16
unit of that term; an emulation of FP32 accumulation shows such entries below
5e-5 of the block maximum at these sizes. Gradients of the zero padding (input
rows >= 24 of W1, output columns >= 3 of W4 and b4) are exactly zero. The Adam
step equals the oracle's on every coordinate whose gradient is not at the noise
level; repeated gradients are bit-identical (fixed-order reductions).
"""
import numpy as np
import pytest
import torch

import paper_1508_02766_amd as K
from oracle import mlp_oracle as N

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _init(seed):
    rng = np.random.default_rng(seed)
    L = []
    for i, (k, n) in enumerate(N.SHAPES):
        W = rng.normal(size=(k, n)) * np.sqrt(2.0 / k)
        b = rng.normal(size=n) * 0.05
        if i == 0:
            W[N.N_IN:, :] = 0
        if i == 3:
            W[:, N.N_OUT:] = 0
            b[N.N_OUT:] = 0
        L.append((W, b))
    return N.pack(L).astype(np.float32).astype(np.float64)


def _data(seed, B):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, N.N_IN)).astype(np.float32)
    T = rng.normal(size=(B, N.N_OUT)).astype(np.float32)
    return X, T


TOL = 2.0 ** -9


def _elementwise(got, ref):
    """Largest entry-wise error relative to the largest reference magnitude."""
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("B", [1, 64, 200, 1000])
def test_forward_matches_oracle(B):
    th = _init(1)
    X, _ = _data(2, B)
    net = K.MlpNet(th)
    Y = net.forward(torch.as_tensor(X, device=DEV)).cpu().numpy()
    y, _ = N.forward(th, X.astype(np.float64))
    assert Y.shape == (B, 3)
    assert _elementwise(Y, y[:, :3]) <= TOL


@pytest.mark.parametrize("B", [37, 256, 1000])
def test_gradient_matches_oracle(B):
    th = _init(3)
    X, T = _data(4, B)
    net = K.MlpNet(th)
    g, loss, _ = net.grad(torch.as_tensor(X, device=DEV), torch.as_tensor(T, device=DEV))
    g = g.cpu().numpy().astype(np.float64)
    lref, gref = N.loss_and_grad(th, X.astype(np.float64), T.astype(np.float64))
    assert float(loss.cpu()[0]) == pytest.approx(lref, rel=1e-4)
    o = 0
    for k, n in N.SHAPES:           # each weight block and bias block separately
        for size in (k * n, n):
            blk, ref = g[o:o + size], gref[o:o + size]
            if np.any(ref != 0):
                assert _elementwise(blk, ref) <= TOL, (k, n, size)
            else:
                assert np.all(blk == 0)
            o += size
    # the zero padding stays out of the gradient exactly
    blocks = N.unpack(g)
    assert np.all(blocks[0][0][N.N_IN:, :] == 0)
    assert np.all(blocks[3][0][:, N.N_OUT:] == 0) and np.all(blocks[3][1][N.N_OUT:] == 0)


def test_gradient_is_deterministic():
    th = _init(5)
    X, T = _data(6, 500)
    net = K.MlpNet(th)
    Xd, Td = torch.as_tensor(X, device=DEV), torch.as_tensor(T, device=DEV)
    g1 = net.grad(Xd, Td)[0]
    g2 = net.grad(Xd, Td)[0]
    assert torch.equal(g1, g2)


def test_adam_step_matches_oracle():
    th = _init(7)
    X, T = _data(8, 300)
    net = K.MlpNet(th)
    lr = 1e-3
    net.train_step(torch.as_tensor(X, device=DEV), torch.as_tensor(T, device=DEV), lr, 1)
    got = net.params()
    _, gref = N.loss_and_grad(th, X.astype(np.float64), T.astype(np.float64))
    ref, _, _ = N.adam(th, gref, np.zeros_like(th), np.zeros_like(th), 1, lr)
    clear = np.abs(gref) > 1e-2 * np.sqrt(np.mean(gref ** 2))
    assert np.max(np.abs(got[clear] - ref[clear])) < 1e-6
    assert np.max(np.abs(got - th)) <= lr * 1.0001 + 1e-7          # a first Adam step moves by at most lr
    pads = N.unpack(got)
    assert np.all(pads[0][0][N.N_IN:, :] == 0) and np.all(pads[3][0][:, N.N_OUT:] == 0)


def test_training_fits_a_smooth_map():
    """200 Adam steps on a fixed smooth regression task cut the loss by 10x."""
    rng = np.random.default_rng(9)
    X = rng.normal(size=(1024, N.N_IN)).astype(np.float32)
    A = rng.normal(size=(N.N_IN, N.N_OUT)) / np.sqrt(N.N_IN)
    T = np.tanh(X @ A).astype(np.float32)
    net = K.MlpNet(_init(10))
    Xd, Td = torch.as_tensor(X, device=DEV), torch.as_tensor(T, device=DEV)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    net.train_step(Xd, Td, 2e-3, 1, loss)
    first = float(loss.cpu()[0])
    for step in range(2, 201):
        net.train_step(Xd, Td, 2e-3, step, loss)
    last = float(loss.cpu()[0])
    assert last < first / 10
