"""Pins of the network oracle (CPU): the FP64 gradient against central finite
differences, the BF16 rounding against torch's own conversion, a hand-sized
forward pass, and the Adam step against torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as N


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    th = rng.normal(size=N.param_count()) * scale
    # padded input rows of W1 and padded output columns of W4 / b4 are zero
    L = N.unpack(th.copy())
    L[0][0][N.N_IN:, :] = 0
    L[3][0][:, N.N_OUT:] = 0
    L[3][1][N.N_OUT:] = 0
    return N.pack(L)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    th = _params(2, 0.2)
    X = rng.normal(size=(9, N.N_IN))
    T = rng.normal(size=(9, N.N_OUT))
    loss, g = N.loss_and_grad(th, X, T, rnd=N.ident)
    idx = rng.choice(th.size, size=60, replace=False)
    for i in idx:
        e = np.zeros_like(th)
        e[i] = 1e-6
        num = (N.loss_and_grad(th + e, X, T, N.ident)[0] - N.loss_and_grad(th - e, X, T, N.ident)[0]) / 2e-6
        assert g[i] == pytest.approx(num, rel=1e-5, abs=1e-8), i


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-20, 20, size=5000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(N.bf16(x), ref)


def test_forward_small_by_hand():
    th = np.zeros(N.param_count())
    L = N.unpack(th)
    L[0][0][0, 0] = 2.0          # z1_0 = 2 x_0 + 1
    L[0][1][0] = 1.0
    L[1][0][0, 1] = -1.0         # z2_1 = -a1_0
    L[1][0][0, 2] = 0.5          # z2_2 = 0.5 a1_0
    L[2][0][2, 0] = 3.0          # z3_0 = 3 a2_2
    L[3][0][0, 2] = 1.0          # y_2 = a3_0 + 0.25
    L[3][1][2] = 0.25
    th = N.pack(L)
    X = np.zeros((2, N.N_IN))
    X[0, 0], X[1, 0] = 1.5, -4.0
    y, _ = N.forward(th, X, N.ident)
    # row 0: a1_0 = 4, a2_2 = 2, a3_0 = 6 -> y_2 = 6.25; row 1: a1_0 = relu(-7) = 0 -> y_2 = 0.25
    assert y[0, 2] == 6.25 and y[1, 2] == 0.25
    assert np.all(y[:, :2] == 0) and np.all(y[:, 3:] == 0)


def test_adam_matches_torch():
    rng = np.random.default_rng(4)
    th = rng.normal(size=50)
    p = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for step in range(1, 6):
        g = rng.normal(size=50)
        p.grad = torch.tensor(g)
        opt.step()
        th, m, v = N.adam(th, g, m, v, step, 1e-2)
    assert np.allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("mutant", ["no_relu_mask", "no_bias_grad", "transposed_W"])
def test_planted_mistakes_are_caught(mutant):
    rng = np.random.default_rng(5)
    th = _params(6, 0.2)
    X = rng.normal(size=(5, N.N_IN))
    T = rng.normal(size=(5, N.N_OUT))
    _, g = N.loss_and_grad(th, X, T, rnd=N.ident)
    L = N.unpack(th)
    y, acts = N.forward(th, X, N.ident)
    B = y.shape[0]
    Tp = np.zeros_like(y)
    Tp[:, :N.N_OUT] = T
    dz = 2.0 * (y - Tp) / B
    grads = [None] * 4
    for i in (3, 2, 1, 0):
        W, _ = L[i]
        gb = dz.sum(axis=0) if mutant != "no_bias_grad" else np.zeros(W.shape[1])
        grads[i] = (acts[i].T @ dz, gb)
        if i > 0:
            Wm = W if mutant != "transposed_W" or W.shape[0] != W.shape[1] else W.T
            da = dz @ Wm.T
            dz = da if mutant == "no_relu_mask" else da * (acts[i] > 0)
    assert np.max(np.abs(N.pack(grads) - g)) > 1e-6 * np.max(np.abs(g))
