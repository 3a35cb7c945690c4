"""The learned-density network on the GPU (BF16 MFMA kernels) against the FP64
oracle (oracle/unet.py).

Layer tests feed the oracle the GPU's own BF16 layer inputs, so each checks one
kernel: forward convolution, input-gradient convolution and weight gradient
(FP32 accumulation of BF16 products; the outputs are rounded once to BF16 with
unit roundoff 2^-9, hence the 4e-3 relative bound on activations).  The
end-to-end test compares the loss, the output and every parameter gradient of
the whole network, where the BF16 rounding of some 30 intermediate tensors
compounds (bounds 3e-2 on r and 6e-2 on each gradient tensor, relative L2).
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import unet as U
from paper_2606_13283_amd import arche

pytestmark = pytest.mark.gpu

GRID = (16, 16, 64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    arche.load()


def bf16(t):
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def params(seed):
    """Oracle parameters with conv weights rounded to BF16 (what the GPU multiplies)."""
    P = U.init_params(seed)
    g = torch.Generator().manual_seed(seed + 1)
    for k in P:
        if k.endswith(".b"):
            P[k] = torch.randn(P[k].shape, dtype=torch.float64, generator=g) * 0.05
        P[k] = P[k].to(torch.float32).to(torch.float64)
        if k.endswith(".w") and P[k].dim() == 5:
            P[k] = bf16(P[k])
    P["out.w"] = P["out.w"] * 4.0
    return P


def flat(P):
    return np.concatenate([P[nm].numpy().reshape(-1) for nm, _ in U.param_shapes()]).astype(np.float32)


def unflat(v):
    out, o = {}, 0
    for nm, shp in U.param_shapes():
        n = int(np.prod(shp))
        out[nm] = torch.tensor(v[o:o + n].astype(np.float64)).reshape(shp)
        o += n
    return out


def fields(seed):
    rng = np.random.default_rng(seed)
    D, H, W = GRID
    z, y, x = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
    n0 = 0.18

    def smooth():
        f = np.zeros(GRID)
        for _ in range(6):
            k = rng.integers(-2, 3, 3)
            f += rng.normal() * np.cos(2 * np.pi * (k[0] * z / D + k[1] * y / H + k[2] * x / W) + rng.uniform(0, 6.3))
        return f

    g = n0 * (1 + 0.3 * np.tanh(smooth()))
    p = n0 * (1 + 0.3 * np.tanh(smooth()))
    c = g * (1 + 0.05 * np.tanh(smooth()))
    return g, p, c, n0


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def to_cf(t):
    """GPU channels-last [D][H][W][C] (numpy) -> oracle [C][D][H][W] (torch f64)."""
    return torch.tensor(np.ascontiguousarray(np.moveaxis(t, -1, 0)), dtype=torch.float64)


@pytest.fixture(scope="module")
def run():
    P = params(11)
    g, p, c, n0 = fields(12)
    net = arche.Net(GRID)
    net.set_params(flat(P))
    loss = net.loss_grad(dev(g), dev(p), dev(c), n0)
    say("gpu loss", loss)
    return net, P, (g, p, c, n0), loss


def close(gpu, ref, rel, what):
    err = np.abs(gpu - ref)
    lim = rel * np.abs(ref) + 1e-3 * np.max(np.abs(ref)) * rel
    bad = err > lim
    assert not bad.any(), (what, int(bad.sum()), float(err.max()), float(np.abs(ref).max()))


def test_param_count_matches_oracle():
    assert arche.load().arche_net_param_count() == U.n_params()


def test_forward_conv_layers(run):
    net, P, _, _ = run
    for l in (0, 1):
        x = to_cf(net.debug(0, 0)) if l == 0 else to_cf(net.debug(3, l))
        ea = to_cf(net.debug(1, l))
        s = to_cf(net.debug(2, l))
        ref_ea = torch.relu(U.conv3(x, P[f"enc{l}.0.w"], P[f"enc{l}.0.b"]))
        ref_s = torch.relu(U.conv3(ea, P[f"enc{l}.1.w"], P[f"enc{l}.1.b"]))
        close(ea.numpy(), ref_ea.numpy(), 4e-3, ("enc0", l))
        close(s.numpy(), ref_s.numpy(), 4e-3, ("enc1", l))
    # decoder level 0: input is up(dout1) + s0
    u0 = to_cf(net.debug(4, 0))
    ref_u0 = U.up(to_cf(net.debug(6, 1))) + to_cf(net.debug(2, 0))
    close(u0.numpy(), ref_u0.numpy(), 4e-3, "up_add")
    da0 = to_cf(net.debug(5, 0))
    close(da0.numpy(), torch.relu(U.conv3(u0, P["dec0.0.w"], P["dec0.0.b"])).numpy(), 4e-3, "dec0.0")
    # pooling
    close(to_cf(net.debug(3, 1)).numpy(), U.pool(to_cf(net.debug(2, 0))).numpy(), 4e-3, "pool")


def conv_vjp(x, w, dz):
    """Oracle input and weight gradients of conv3 for output gradient dz."""
    xx = x.clone().requires_grad_(True)
    ww = w.clone().requires_grad_(True)
    y = U.conv3(xx, ww, torch.zeros(w.shape[0], dtype=torch.float64))
    gx, gw = torch.autograd.grad(y, (xx, ww), dz)
    return gx, gw, dz.sum(dim=(1, 2, 3))


def test_backward_conv_layers(run):
    net, P, _, _ = run
    G = unflat(net.grads())
    for l in (0, 1):
        ds = to_cf(net.debug(9, l))       # grad of s[l] (skip + pooled path)
        s = to_cf(net.debug(2, l))
        ea = to_cf(net.debug(1, l))
        x = to_cf(net.debug(0, 0)) if l == 0 else to_cf(net.debug(3, l))
        dz1 = ds * (s > 0)
        gx1, gw1, gb1 = conv_vjp(ea, P[f"enc{l}.1.w"], dz1)
        gB = to_cf(net.debug(8, l))
        close(gB.numpy(), gx1.numpy(), 4e-3, ("dgrad enc1", l))
        assert torch.allclose(G[f"enc{l}.1.w"], gw1, rtol=1e-3, atol=1e-4 * float(gw1.abs().max())), l
        assert torch.allclose(G[f"enc{l}.1.b"], gb1, rtol=1e-3, atol=1e-4 * float(gb1.abs().max())), l
        dz0 = gB * (ea > 0)
        gx0, gw0, gb0 = conv_vjp(x, P[f"enc{l}.0.w"], dz0)
        close(to_cf(net.debug(7, l)).numpy(), gx0.numpy(), 4e-3, ("dgrad enc0", l))
        assert torch.allclose(G[f"enc{l}.0.w"], gw0, rtol=1e-3, atol=1e-4 * float(gw0.abs().max())), l


def test_end_to_end_against_oracle(run):
    net, P, (g, p, c, n0), loss = run
    x = U.inputs(g, p, n0)
    t = U.target(c, p, n0)
    L_ref, G_ref = U.loss_and_grads(P, x, t)
    r_ref = U.forward(P, x).numpy()
    r = torch.empty(GRID, dtype=torch.float64, device="cuda")
    net.forward(dev(g), dev(p), n0, r)
    torch.cuda.synchronize()
    r = r.cpu().numpy()
    er = np.linalg.norm(r - r_ref) / np.linalg.norm(r_ref)
    say("loss gpu %.6e oracle %.6e; r rel err %.2e" % (loss, L_ref, er))
    assert er <= 3e-2
    assert abs(loss - L_ref) <= 3e-2 * L_ref
    G = unflat(net.grads())
    num = den = 0.0
    for nm, _ in U.param_shapes():
        a, b = G[nm].reshape(-1), G_ref[nm].reshape(-1)
        e = float(torch.linalg.norm(a - b) / max(float(torch.linalg.norm(b)), 1e-30))
        say("grad", nm, "rel err %.2e" % e)
        assert e <= 6e-2, (nm, e)
        num += float(a @ b)
        den += float(torch.linalg.norm(a) * torch.linalg.norm(b))
    assert num / den >= 0.999


def test_training_lowers_the_loss():
    P = params(21)
    g, p, c, n0 = fields(22)
    net = arche.Net(GRID)
    net.set_params(flat(P))
    gd, pd, cd = dev(g), dev(p), dev(c)
    first = net.loss_grad(gd, pd, cd, n0)
    for _ in range(30):
        net.adam_step(1e-3)
        last = net.loss_grad(gd, pd, cd, n0)
    say("loss %.3e -> %.3e" % (first, last))
    assert last < 0.5 * first
    net.close()


def test_net_rejects_bad_grids():
    with pytest.raises(arche.ArcheError):
        arche.Net((16, 16, 20))
    with pytest.raises(arche.ArcheError):
        arche.Net((8, 8, 8))
