"""Pins of the U-Net oracle (oracle/unet.py) against definitions written out
here independently: brute-force periodic convolution, block mean and nearest
copy, the pool/up adjoint identity, the parameter count, periodic translation
equivariance, and FP64 central finite differences of the whole network."""
import numpy as np
import pytest
import torch

from oracle import unet as U


def brute_conv3(x, w, b):
    C, D, H, W = x.shape
    O = w.shape[0]
    out = np.zeros((O, D, H, W))
    for o in range(O):
        for d in range(D):
            for h in range(H):
                for q in range(W):
                    s = b[o]
                    for i in range(C):
                        for a in range(3):
                            for c in range(3):
                                for e in range(3):
                                    s += w[o, i, a, c, e] * x[i, (d + a - 1) % D, (h + c - 1) % H, (q + e - 1) % W]
                    out[o, d, h, q] = s
    return out


def test_conv3_matches_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 4, 3, 5))
    w = rng.normal(size=(3, 2, 3, 3, 3))
    b = rng.normal(size=3)
    got = U.conv3(torch.tensor(x), torch.tensor(w), torch.tensor(b)).numpy()
    assert np.allclose(got, brute_conv3(x, w, b), rtol=1e-13, atol=1e-12)


def test_conv1_matches_definition():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 2, 4, 2))
    w = rng.normal(size=(5, 2))
    b = rng.normal(size=5)
    got = U.conv1(torch.tensor(x), torch.tensor(w), torch.tensor(b)).numpy()
    ref = np.zeros((5, 2, 4, 2))
    for o in range(5):
        ref[o] = b[o] + w[o, 0] * x[0] + w[o, 1] * x[1]
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-14)


def test_pool_up_definitions_and_adjoint():
    rng = np.random.default_rng(2)
    y = rng.normal(size=(3, 4, 6, 8))
    p = U.pool(torch.tensor(y)).numpy()
    ref = y.reshape(3, 2, 2, 3, 2, 4, 2).mean(axis=(2, 4, 6))
    assert np.allclose(p, ref, rtol=1e-14, atol=1e-15)
    x = rng.normal(size=(3, 2, 3, 4))
    u = U.up(torch.tensor(x)).numpy()
    for d in range(4):
        for h in range(6):
            for q in range(8):
                assert np.array_equal(u[:, d, h, q], x[:, d // 2, h // 2, q // 2])
    lhs = np.sum(u * y)
    rhs = 8.0 * np.sum(x * p)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_param_count():
    assert U.N_CONV3 == 14
    assert U.n_params() == 2 * 32 + 32 + 14 * (27 * 32 * 32 + 32) + 32 + 1 == 387649


def test_translation_equivariance():
    """A periodic shift by 8 points (a whole coarsest cell) shifts the output."""
    P = U.init_params(3)
    for k in P:
        if k.endswith(".b"):
            P[k] = torch.randn(P[k].shape, dtype=torch.float64) * 0.1
    x = torch.randn(2, 16, 8, 8, dtype=torch.float64, generator=torch.Generator().manual_seed(4))
    r = U.forward(P, x)
    r2 = U.forward(P, torch.roll(x, shifts=8, dims=1))
    assert torch.allclose(torch.roll(r, shifts=8, dims=0), r2, rtol=1e-12, atol=1e-13)


def test_gradients_match_finite_differences():
    P = U.init_params(5)
    g = torch.Generator().manual_seed(6)
    for k in P:
        if k.endswith(".b"):
            P[k] = torch.randn(P[k].shape, dtype=torch.float64, generator=g) * 0.05
    P["out.w"] = P["out.w"] * 10.0
    x = torch.randn(2, 8, 8, 8, dtype=torch.float64, generator=g)
    t = torch.randn(8, 8, 8, dtype=torch.float64, generator=g) * 0.1
    L0, G = U.loss_and_grads(P, x, t)
    rng = np.random.default_rng(7)
    h = 1e-6
    checked = 0
    for k in P:
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.numel(), size=min(3, flat.numel()), replace=False):
            old = float(flat[idx])
            flat[idx] = old + h
            Lp = float(U.loss(P, x, t))
            flat[idx] = old - h
            Lm = float(U.loss(P, x, t))
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            an = float(G[k].reshape(-1)[idx])
            assert abs(fd - an) <= 2e-5 * max(abs(fd), 1e-4 * abs(L0)) + 1e-12, (k, int(idx), fd, an)
            checked += 1
    assert checked >= 60
