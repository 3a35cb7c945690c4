"""Training and evaluation driver of the learned initial density (arche_net.h).

Samples come from the method itself: an MD trajectory with the plain
(one-center) guess, where each step records, at the new positions, the guide
G = n0 + the one-center superposition's change since the previous step, the
previous converged density p and the converged density n.  The network learns
r = n/n0 - 1 - (p/n0 - 1), the converged density's change, from [G, p].  Every numerical
step runs in the library's kernels; this module only sequences the calls and
keeps the samples in device memory (torch tensors).
"""
from __future__ import annotations

import numpy as np
import torch

from . import arche


def param_layout():
    """(name, shape) of every parameter in the library's order (arche_net.h)."""
    out = [("in.w", (32, 2)), ("in.b", (32,))]
    names = ["enc%d.%d" % (l, j) for l in range(4) for j in range(2)]
    names += ["dec%d.%d" % (l, j) for l in (2, 1, 0) for j in range(2)]
    for nm in names:
        out += [(nm + ".w", (32, 32, 3, 3, 3)), (nm + ".b", (32,))]
    return out + [("out.w", (1, 32)), ("out.b", (1,))]


def init_params(seed):
    """He-normal weights (fan-in scaled), zero biases, a small output layer."""
    rng = np.random.default_rng(seed)
    parts = []
    for nm, shp in param_layout():
        if nm.endswith(".b"):
            parts.append(np.zeros(int(np.prod(shp))))
        else:
            fan_in = int(np.prod(shp[1:]))
            scale = np.sqrt(2.0 / fan_in) * (0.1 if nm == "out.w" else 1.0)
            parts.append(rng.normal(0.0, scale, int(np.prod(shp))))
    return np.concatenate(parts).astype(np.float32)


def _opts(w, init, tol=1e-10):
    return arche.Options(w_fixed=w.w_fixed, lambda_vw=w.lam, xc=arche.XC_LDA if w.xc else arche.XC_NONE,
                         init=init, scf_tol=tol)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


class Trajectory:
    """Verlet MD (Sec. 2.1) through the library (arche_md_step); before a step,
    the learned proposal's guide at the next positions can be recorded
    (arche_md_predict, arche_learned_guide), for training samples."""

    def __init__(self, w, init=arche.INIT_ONE_CENTER, net=None, tol=1e-10):
        self.w = w
        self.ctx = arche.Context.from_workload(w, _opts(w, init, tol))
        if net is not None:
            self.ctx.set_init_net(net)
        self.pos = w.pos.copy()
        self.vel = (w.vel if w.vel is not None else np.zeros_like(self.pos)).copy()
        self.res = self.ctx.solve(self.pos)

    def next_positions(self):
        return self.ctx.md_predict(self.w.dt, self.pos, self.vel)

    def step(self, record=False):
        """One MD step; returns (result, sample or None), the sample being
        (guide G, previous converged density, converged density) on the device."""
        sample = None
        if record:
            p = self.ctx.density()
            g = self.ctx.learned_guide(self.next_positions())
        self.pos, self.vel, _, res = self.ctx.md_step(self.w.dt, self.pos, self.vel)
        if record:
            sample = (_dev(g), _dev(p), _dev(self.ctx.density()))
        self.res = res
        return res, sample

    def solve_at(self, pos):
        """A solve at given positions (another trajectory's), with this
        context's initial density."""
        self.pos = np.array(pos, dtype=np.float64)
        self.res = self.ctx.solve(self.pos)
        return self.res

    def close(self):
        self.ctx.close()


def generate(workloads, steps):
    """Samples (g, p, n) from `steps` plain MD steps of each workload."""
    out = []
    for w in workloads:
        tr = Trajectory(w)
        for _ in range(steps):
            _, s = tr.step(record=True)
            if s is not None:
                out.append((s, w.cell))
        tr.close()
    return out


def n0_of(w):
    return float(np.sum([w.Z[s] for s in w.species])) / float(np.prod(w.cell))


def train(net, samples, n0s, epochs, lr=1e-3, seed=0, lr_end=1e-4):
    """Adam over the samples (seeded order), learning rate decayed geometrically
    from lr to lr_end.  Returns the mean loss of each epoch."""
    rng = np.random.default_rng(seed)
    hist = []
    total = epochs * len(samples)
    k = 0
    for _ in range(epochs):
        order = rng.permutation(len(samples))
        acc = 0.0
        for i in order:
            g, p, n = samples[i]
            acc += net.loss_grad(g, p, n, n0s[i])
            rate = lr * (lr_end / lr) ** (k / max(total - 1, 1))
            net.adam_step(rate)
            k += 1
        hist.append(acc / len(samples))
    return hist


def compare(w, net, steps):
    """The plain guess (one-center, uniform where it rings negative), the
    previous converged density alone (what an untrained network proposes) and
    the learned proposal, solved at the same positions: the plain trajectory
    drives the positions, the others follow it, one after another with only
    their own context alive.  Per-step SCF iterations and free energies."""
    rows = [dict() for _ in range(steps)]
    positions = []
    plain = Trajectory(w)
    for k in range(steps):
        a, _ = plain.step()
        positions.append(plain.pos.copy())
        rows[k].update(plain_iters=a["scf_iters"], plain_fallback=a["used_fallback"], F_plain=a["F"])
    plain.close()
    prev = Trajectory(w, init=arche.INIT_KEEP)
    for k in range(steps):
        prev.ctx.set_density(prev.ctx.density())
        c = prev.solve_at(positions[k])
        rows[k].update(prev_iters=c["scf_iters"], F_prev=c["F"])
    prev.close()
    learned = Trajectory(w, init=arche.INIT_LEARNED, net=net)
    for k in range(steps):
        b = learned.solve_at(positions[k])
        rows[k].update(learned_iters=b["scf_iters"], F_learned=b["F"], fallback=b["used_fallback"])
    learned.close()
    return rows
