"""Oracle (test infrastructure only): the learned initial-density network in
plain FP64 PyTorch on the CPU, the reference the GPU's BF16 kernels are checked
against.  Only tests may import it.

The paper's initial densities (Sec. 2.5, 2.5.1) are the uniform one and the
one-center profile; the learned proposal is an addition that replaces the
one-center guess: the previous converged density p moved by the change the
network predicts from p and from the one-center superposition's own change
between the old and the new positions.  The network is a 3D U-Net on the periodic
grid, constant width 32 on four levels:

  x = [a, b] with a = G/n0 - 1 (G = n0 + the superposition's change
      g^ (S_Z(new) - S_Z(old)) transformed to real space), b = p/n0 - 1,
      n0 = N_e/|Omega|
  h = relu(conv1(x; 2->32))
  s0 = E0(h)                      E_l = two (conv3 32->32, relu)      level 0
  s1 = E1(pool(s0)), s2 = E2(pool(s1)), z = E3(pool(s2))             levels 1-3
  d2 = D2(up(z) + s2), d1 = D1(up(d2) + s1), d0 = D0(up(d1) + s0)    D_l like E_l
  r = conv1(d0; 32->1)
  proposal n = p + n0 LP(r)  (LP: low pass exp(-(|k|/k_c)^2), k_c a quarter of
           the Nyquist frequency; then floored at 0.1 p and renormalised)

conv3: 3x3x3 cross-correlation with periodic wrap (the cell is periodic) and a
bias; conv1: 1x1x1 with bias; pool: mean over 2x2x2 blocks; up: nearest
(each coarse value copied to its 8 fine points).  Loss: mean over the grid of
(r - r*)^2 with r* = n_conv/n0 - 1 - b: the network learns the converged
density's change from the previous step, guided by the superposition's change
(the low pass keeps the short-wavelength part of its error out of the guess,
where it slows the SCF down).  Parameters: 2*32+32 + 14*(27*32*32+32)
+ 32+1 = 387,649.

Pins (tests/test_oracle_unet.py): conv3 against a brute-force loop sum on
small grids; pool/up against their definitions and the adjoint identity
<up(x), y> = 8 <x, pool(y)>; the parameter count; the whole network's gradient
against central finite differences in FP64.  The trained network's output has
no closed form: "parity unpinned" for what it predicts (it is judged by the SCF
iterations it saves at an unchanged converged answer).
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as Fn

WIDTH = 32
LEVELS = 4
N_CONV3 = 2 * LEVELS + 2 * (LEVELS - 1)  # 14


def conv3(x, w, b):
    """Periodic 3x3x3 cross-correlation: out[o, p] = b[o] + sum_{i, t} w[o, i, t] x[i, p + t - 1].
    x: [C_in, D, H, W]; w: [C_out, C_in, 3, 3, 3]; b: [C_out]."""
    xp = Fn.pad(x[None], (1, 1, 1, 1, 1, 1), mode="circular")
    return Fn.conv3d(xp, w, b)[0]


def conv1(x, w, b):
    """1x1x1 convolution: out[o, p] = b[o] + sum_i w[o, i] x[i, p]. w: [C_out, C_in]."""
    return torch.einsum("oi,idhw->odhw", w, x) + b[:, None, None, None]


def pool(x):
    """Mean over 2x2x2 blocks."""
    return Fn.avg_pool3d(x[None], 2)[0]


def up(x):
    """Nearest upsampling by 2 in each direction."""
    return x.repeat_interleave(2, 1).repeat_interleave(2, 2).repeat_interleave(2, 3)


def param_shapes():
    """Ordered (name, shape) of every parameter."""
    out = [("in.w", (WIDTH, 2)), ("in.b", (WIDTH,))]
    names = [f"enc{l}.{j}" for l in range(LEVELS) for j in range(2)]
    names += [f"dec{l}.{j}" for l in range(LEVELS - 2, -1, -1) for j in range(2)]
    for nm in names:
        out += [(nm + ".w", (WIDTH, WIDTH, 3, 3, 3)), (nm + ".b", (WIDTH,))]
    out += [("out.w", (1, WIDTH)), ("out.b", (1,))]
    return out


def n_params():
    return int(sum(np.prod(s) for _, s in param_shapes()))


def init_params(seed, dtype=torch.float64):
    """He-normal weights, zero biases; out.w scaled down so the initial r is small."""
    g = torch.Generator().manual_seed(seed)
    P = {}
    for nm, shp in param_shapes():
        if nm.endswith(".b"):
            P[nm] = torch.zeros(shp, dtype=dtype)
        else:
            fan_in = int(np.prod(shp[1:]))
            std = (2.0 / fan_in) ** 0.5 * (0.1 if nm == "out.w" else 1.0)
            P[nm] = torch.randn(shp, generator=g, dtype=dtype) * std
    return P


def forward(P, x):
    """x: [2, D, H, W] (D, H, W divisible by 8).  Returns r: [D, H, W]."""
    def block(h, nm):
        h = torch.relu(conv3(h, P[nm + ".0.w"], P[nm + ".0.b"]))
        return torch.relu(conv3(h, P[nm + ".1.w"], P[nm + ".1.b"]))

    h = torch.relu(conv1(x, P["in.w"], P["in.b"]))
    skips = []
    for l in range(LEVELS):
        if l > 0:
            h = pool(h)
        h = block(h, f"enc{l}")
        skips.append(h)
    for l in range(LEVELS - 2, -1, -1):
        h = block(up(h) + skips[l], f"dec{l}")
    return conv1(h, P["out.w"], P["out.b"])[0]


def loss(P, x, r_target):
    r = forward(P, x)
    return torch.mean((r - r_target) ** 2)


def loss_and_grads(P, x, r_target):
    """FP64 loss and d loss / d parameter for every parameter (autograd on the CPU)."""
    Q = {k: v.detach().clone().requires_grad_(True) for k, v in P.items()}
    L = loss(Q, x, r_target)
    L.backward()
    return float(L), {k: Q[k].grad.detach() for k in Q}


def inputs(n_guess, n_prev, n0):
    """Network input from the guide field G and the previous converged density."""
    return torch.stack([torch.as_tensor(n_guess) / n0 - 1.0, torch.as_tensor(n_prev) / n0 - 1.0])


def target(n_conv, n_prev, n0):
    return torch.as_tensor(n_conv) / n0 - 1.0 - (torch.as_tensor(n_prev) / n0 - 1.0)
