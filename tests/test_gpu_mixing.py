"""More's weight exactly as printed (Sec. 2.5.2: U the Hartree interaction of
dn with itself, K = int dn^2 / (dn_a/dmu)) on the GPU against the oracle's
SCF loop, iteration by iteration (residuals and weights), and the converged
answer equal to that of the default (secant) weight."""
import sys

import numpy as np
import pytest

from oracle import md as omd
from oracle import scf as oscf
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


def cell():
    w = W.small_random(8, 20, 2.7, 5.0, seed=12)
    w.lam = 0.0  # Thomas-Fermi + Hartree + xc
    return w


def test_printed_weight_iterations_match_oracle():
    w = cell()
    its = 12
    o = arche.Options(w_fixed=w.w_fixed, lambda_vw=0.0, xc=arche.XC_LDA, init=arche.INIT_UNIFORM, scf_tol=1e-300,
                      scf_max_iter=its, mixing=arche.MIX_MORE_PRINTED, more_warmup=2, more_trust=1e30)
    ctx = arche.Context.from_workload(w, o)
    ctx.solve(w.pos, allow_noconv=True)
    h = ctx.history()
    ctx.close()
    s = oscf.System(w.cell, w.grid, w.pos, w.species, w.Z, w.rc, w.mass, w.kT, 0.0, True)
    ion = oscf.ionic_setup(s)
    r = oscf.scf(s, ion, oscf.initial_density(s, ion)[0], mixing="more_printed", tol=1e-300, max_iter=its,
                 warmup=2, w_fixed=w.w_fixed, more_trust=1e30)
    say("weights gpu", h[:, 2], "oracle", r.weights)
    for t in range(its):
        assert abs(h[t, 1] - r.history[t]) <= 1e-9 * r.history[t], (t, h[t, 1], r.history[t])
    for t in range(its - 1):
        assert abs(h[t, 2] - r.weights[t]) <= 1e-9, (t, h[t, 2], r.weights[t])
    assert any(abs(x - w.w_fixed) > 1e-3 for x in r.weights[2:its - 1])  # More's own weight was taken


def test_printed_weight_same_fixed_point():
    w = cell()
    res = {}
    for name, mix in (("printed", arche.MIX_MORE_PRINTED), ("secant", arche.MIX_MORE)):
        o = arche.Options(w_fixed=w.w_fixed, lambda_vw=0.0, xc=arche.XC_LDA, init=arche.INIT_UNIFORM,
                          scf_tol=1e-12, mixing=mix)
        ctx = arche.Context.from_workload(w, o)
        res[name] = ctx.solve(w.pos)
        ctx.close()
        say(name, res[name]["scf_iters"], res[name]["F"])
    assert abs(res["printed"]["F"] - res["secant"]["F"]) <= 1e-11 * abs(res["secant"]["F"])
    assert abs(res["printed"]["P"] - res["secant"]["P"]) <= 1e-10 * abs(res["secant"]["P"])
