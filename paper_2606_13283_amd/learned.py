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
    """Verlet MD (Sec. 2.1) driven from Python around Context.solve, so that the
    guess for the next step can be recorded before the solve."""

    def __init__(self, w, init=arche.INIT_ONE_CENTER, net=None, tol=1e-10):
        self.w = w
        self.ctx = arche.Context.from_workload(w, _opts(w, init, tol))
        if net is not None:
            self.ctx.set_init_net(net)
        self.m = np.array([w.mass[s] for s in w.species])[:, None]
        self.r = w.pos.copy()
        self.res = self.ctx.solve(self.r)
        self.F = self.ctx.forces()
        v = w.vel if w.vel is not None else np.zeros_like(self.r)
        self.r_prev = self.r - v * w.dt + self.F * w.dt ** 2 / (2 * self.m)

    def next_positions(self):
        return 2 * self.r - self.r_prev + self.F * self.w.dt ** 2 / self.m

    def step(self, r_next=None, record=False):
        """One step; returns (result, sample or None)."""
        r_next = self.next_positions() if r_next is None else r_next
        sample = None
        if record:
            p = self.ctx.density()
            _, _, g = self.ctx.one_center_raw(r_next)
        res = self.ctx.solve(r_next)
        if record:
            sample = (_dev(g), _dev(p), _dev(self.ctx.density()))
        self.r_prev, self.r = self.r, r_next
        self.F = self.ctx.forces()
        self.res = res
        return res, sample

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
    drives the positions, the others follow it.  Per-step SCF iterations and
    free energies."""
    plain = Trajectory(w)
    prev = Trajectory(w, init=arche.INIT_KEEP)
    learned = Trajectory(w, init=arche.INIT_LEARNED, net=net)
    rows = []
    for _ in range(steps):
        r_next = plain.next_positions()
        a, _ = plain.step(r_next)
        prev.ctx.set_density(prev.ctx.density())
        c, _ = prev.step(r_next)
        b, _ = learned.step(r_next)
        rows.append({"plain_iters": a["scf_iters"], "plain_fallback": a["used_fallback"],
                     "prev_iters": c["scf_iters"], "learned_iters": b["scf_iters"], "F_plain": a["F"],
                     "F_prev": c["F"], "F_learned": b["F"], "fallback": b["used_fallback"]})
    for t in (plain, prev, learned):
        t.close()
    return rows
