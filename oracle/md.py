"""Oracle (test infrastructure only): Verlet molecular dynamics, Sec. 2.1, and
a whole-step driver that chains structure factor, initial density, SCF, forces.

Position Verlet (Sec. 2.1):
  r(t + dt) = 2 r(t) - r(t - dt) + F(t)/m dt^2
  v(t)      = (r(t + dt) - r(t - dt)) / (2 dt)
(the printed velocity formula has '+', a misprint: the central difference has
'-').  Start: r(-dt) = r(0) - v(0) dt + F(0) dt^2 / (2 m) (second-order Taylor
step; the paper does not say how the first step starts).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import scf as scf_mod
from . import thermo


def masses(sys: scf_mod.System) -> np.ndarray:
    return np.array([sys.mass[s] for s in sys.species])


def verlet_start(r0, v0, F0, m, dt):
    return r0 - v0 * dt + F0 * dt * dt / (2.0 * m[:, None])


def verlet_step(r, r_prev, F, m, dt):
    r_next = 2.0 * r - r_prev + F * dt * dt / m[:, None]
    v = (r_next - r_prev) / (2.0 * dt)
    return r_next, v


@dataclass
class StepResult:
    sys: scf_mod.System
    ion: scf_mod.Ionic
    scf: scf_mod.SCFResult
    th: thermo.Thermo
    nhat: np.ndarray


def solve_at(sys, init="uniform", prev=None, mixing="more", tol=1e-10, mu0=None,
             max_iter=2000, solver="paper") -> StepResult:
    """Structure factor -> V^ie -> initial density -> SCF -> F, P, forces.
    solver "paper": the iteration of Sec. 2.5 (`scf`); "anderson": the same
    fixed point by `scf_anderson` (for tests that only need the solution)."""
    ion = scf_mod.ionic_setup(sys)
    n0, fb = scf_mod.initial_density(sys, ion, init, prev)
    if solver == "anderson":
        res = scf_mod.scf_anderson(sys, ion, n0, tol=tol, max_iter=max_iter, beta=0.3, mu0=mu0)
    else:
        res = scf_mod.scf(sys, ion, n0, mixing=mixing, tol=tol, mu0=mu0, max_iter=max_iter)
    res.used_fallback = fb
    th = thermo.evaluate(sys, ion, res)
    return StepResult(sys, ion, res, th, sys.grid.forward(res.n))
