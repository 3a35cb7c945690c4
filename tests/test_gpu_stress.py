"""The stress tensor of Sec. 2.6 on the GPU (arche_stress) against the
oracle's, term by term and element by element, on an orthorhombic one-species
cell with ion velocities and on a two-species cell; and the trace against the
pressure of the same solve."""
import math
import sys

import numpy as np
import pytest

from oracle import md as omd
from oracle import scf as oscf
from oracle import stress as ostress
from paper_2606_13283_amd import arche
from paper_2606_13283_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    arche.load()


def ortho():
    return W.small_random(6, 16, 2.7, 8.0, seed=17, shape=(16, 18, 20), stretch=(0.9, 1.0, 1.15))


def two_species():
    w = W.small_random(10, 16, 2.7, 8.0, seed=3, shape=(16, 20, 24), stretch=(1.0, 1.2, 1.4))
    w.species = np.array([0, 1] * 5, dtype=np.int32)
    w.Z, w.rc, w.mass = (3.0, 1.0), (1.1, 0.6), (W.AL_MASS, 1837.0)
    return w


@pytest.mark.parametrize("mk", [ortho, two_species])
def test_stress_terms_match_oracle(mk):
    w = mk()
    say("stress", w.name)
    vel = np.random.default_rng(9).normal(0, math.sqrt(w.kT / W.AL_MASS), w.pos.shape)
    o = arche.Options(w_fixed=w.w_fixed, lambda_vw=w.lam, xc=arche.XC_LDA, init=arche.INIT_UNIFORM, scf_tol=1e-12)
    ctx = arche.Context.from_workload(w, o)
    res = ctx.solve(w.pos)
    assert res["converged"]
    sig, terms = ctx.stress(vel)
    ctx.close()
    s = oscf.System(w.cell, w.grid, w.pos, w.species, w.Z, w.rc, w.mass, w.kT, w.lam, w.xc)
    ref = omd.solve_at(s, tol=1e-12)
    T = ostress.stress(s, ref.ion, ref.scf, vel=vel)
    tot = ostress.total(T)
    scale = np.max(np.abs(tot))
    for k in ostress.TERMS:
        err = np.max(np.abs(terms[k] - T[k]))
        assert err <= 1e-9 * max(np.max(np.abs(T[k])), 1e-3 * scale), (k, terms[k], T[k])
    assert np.max(np.abs(sig - tot)) <= 1e-9 * scale
    # without the ions' kinetic term the trace is the pressure (Ewald part to truncation)
    P = -np.trace(sig - terms["i"]) / 3.0
    assert abs(P - res["P"]) <= 1e-5 * abs(res["P"])
    # off-diagonal entries are present
    assert np.max(np.abs(sig - np.diag(np.diag(sig)))) > 1e-3 * scale
