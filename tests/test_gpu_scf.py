"""GPU parity of the whole SCF path against the oracle: small cells solved by
both sides (element-wise density, mu, energy terms, pressure, forces), the
one-center guess, MD steps, determinism and error paths; and the full-size
workloads through properties and samples the oracle can compute."""
import math
import sys

import numpy as np
import pytest

from oracle import fd as ofd
from oracle import ionic as oion
from oracle import md as omd
from oracle import scf as oscf
from oracle import thermo as oth
from paper_2606_13283_amd import arche
from paper_2606_13283_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-9  # free energy, pressure and forces


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    arche.load()


def system_of(w):
    return oscf.System(w.cell, w.grid, w.pos, w.species, w.Z, w.rc, w.mass, w.kT, w.lam, w.xc)


def opts_of(w, **kw):
    o = arche.Options(w_fixed=w.w_fixed, lambda_vw=w.lam, xc=arche.XC_LDA if w.xc else arche.XC_NONE)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


FORCE_ZERO = 1e-12  # forces that vanish by symmetry are compared as zero (rounding level)


def force_err(Fg, Fo):
    """max |F_gpu - F_oracle| relative to max |F_oracle|; where the oracle's forces are
    at rounding level (a perfect lattice) both sides must be below FORCE_ZERO."""
    if np.max(np.abs(Fo)) < 1e3 * FORCE_ZERO:
        return 0.0 if max(np.max(np.abs(Fg)), np.max(np.abs(Fo))) <= FORCE_ZERO else np.inf
    return np.max(np.abs(Fg - Fo)) / np.max(np.abs(Fo))


def check_against(res, Fg, ref_th, ref_mu, label):
    assert abs(res["F"] - ref_th.F) <= RTOL * abs(ref_th.F), (label, res["F"], ref_th.F)
    assert abs(res["P"] - ref_th.P) <= RTOL * abs(ref_th.P), (label, res["P"], ref_th.P)
    assert abs(res["E"] - ref_th.E) <= RTOL * abs(ref_th.E), label
    for k in ("F_TF", "F_vW", "E_H", "F_xc", "E_ie", "U_ii"):
        scale = max(abs(ref_th.terms[k]), 1e-3 * abs(ref_th.F))
        assert abs(res["terms"][k] - ref_th.terms[k]) <= RTOL * scale, (label, k, res["terms"][k], ref_th.terms[k])
    for k in ref_th.P_terms:
        scale = max(abs(ref_th.P_terms[k]), 1e-3 * abs(ref_th.P))
        assert abs(res["P_terms"][k] - ref_th.P_terms[k]) <= RTOL * scale, (label, k)
    assert abs(res["mu"] - ref_mu) <= RTOL * max(abs(ref_mu), 1e-3), label
    assert force_err(Fg, ref_th.forces) <= RTOL, (label, force_err(Fg, ref_th.forces))


SMALL = {
    "rand4_16c_10eV": lambda: W.small_random(4, 16, 2.7, 10.0, seed=11),
    "rand8_20c_5eV": lambda: W.small_random(8, 20, 2.7, 5.0, seed=12),
    "ortho2sp_16x20x24": None,
}


def two_species():
    w = W.small_random(10, 16, 2.7, 8.0, seed=3, shape=(16, 20, 24), stretch=(1.0, 1.2, 1.4))
    w.species = np.array([0, 1] * 5, dtype=np.int32)
    w.Z, w.rc, w.mass = (3.0, 1.0), (1.1, 0.6), (W.AL_MASS, 1837.0)
    return w


@pytest.fixture(scope="module")
def small_solved():
    out = {}
    for name, mk in SMALL.items():
        w = mk() if mk else two_species()
        say("oracle solve", name)
        s = system_of(w)
        r = omd.solve_at(s, tol=1e-12)
        assert r.scf.converged
        out[name] = (w, r)
    return out


@pytest.mark.parametrize("name", list(SMALL))
def test_small_cell_parity(small_solved, name):
    w, r = small_solved[name]
    say("gpu solve", name)
    ctx = arche.Context.from_workload(w, opts_of(w, scf_tol=1e-12, init=arche.INIT_UNIFORM))
    res = ctx.solve(w.pos)
    assert res["converged"]
    Fg = ctx.forces()
    n = ctx.density()
    assert np.max(np.abs(n - r.scf.n)) <= 1e-9 * np.max(r.scf.n)
    check_against(res, Fg, r.th, r.scf.mu, name)
    # iteration counts follow the same algorithm (rounding may shift the last one)
    assert abs(res["scf_iters"] - r.scf.iters) <= 2, (res["scf_iters"], r.scf.iters)
    ctx.close()


def test_one_center_guess_parity(small_solved):
    w, r = small_solved["rand4_16c_10eV"]
    ctx = arche.Context.from_workload(w, opts_of(w, scf_tol=1e-12))
    ctx.solve(w.pos)
    n_gpu = ctx.density()
    rng = np.random.default_rng(1)
    new = w.pos + rng.normal(0, 0.05, w.pos.shape)
    guess, fb = ctx.one_center_guess(new)
    s = system_of(w)
    g = s.grid
    prev = (g.forward(n_gpu), oion.charge_structure_factor(
        oion.structure_factors(g, w.pos, w.species, 1), w.Z))
    s2 = s.with_positions(new)
    ref, fb_ref = oscf.initial_density(s2, oscf.ionic_setup(s2), "one_center", prev)
    assert fb == fb_ref
    assert np.max(np.abs(guess - ref)) <= 1e-11 * np.max(ref)
    ctx.close()


def test_md_steps_parity(small_solved):
    w, r = small_solved["rand4_16c_10eV"]
    ctx = arche.Context.from_workload(w, opts_of(w, scf_tol=1e-12))
    rng = np.random.default_rng(2)
    vel = rng.normal(0, math.sqrt(w.kT / W.AL_MASS), w.pos.shape)
    pos = w.pos.copy()
    ctx.solve(pos)
    F0 = ctx.forces()
    m = np.full(4, W.AL_MASS)
    dt = 4 * W.DT_02FS
    r_prev = omd.verlet_start(pos, vel, F0, m, dt)
    r_cur, Fc = pos, F0
    s = system_of(w)
    for step in range(2):
        say("md step", step)
        pos_n, vel_n, F, res = ctx.md_step(dt, pos, vel)
        r_next, v_ref = omd.verlet_step(r_cur, r_prev, Fc, m, dt)
        assert np.max(np.abs(pos_n - r_next)) <= 1e-13 * np.max(np.abs(r_next))
        assert np.max(np.abs(vel_n - v_ref)) <= 1e-12 * np.max(np.abs(v_ref))
        ro = omd.solve_at(s.with_positions(pos_n), tol=1e-12)
        check_against(res, F, ro.th, ro.scf.mu, "md%d" % step)
        r_prev, r_cur, Fc = r_cur, r_next, F
        pos, vel = pos_n, vel_n
    ctx.close()


def test_deterministic_and_fixed_mixing(small_solved):
    w, r = small_solved["rand4_16c_10eV"]
    ctx = arche.Context.from_workload(w, opts_of(w, scf_tol=1e-12, init=arche.INIT_UNIFORM))
    a = ctx.solve(w.pos)
    na = ctx.density()
    b = ctx.solve(w.pos)
    nb = ctx.density()
    assert a["F"] == b["F"] and a["P"] == b["P"] and np.array_equal(na, nb)
    ctx.close()
    ctx = arche.Context.from_workload(w, opts_of(w, scf_tol=1e-12, init=arche.INIT_UNIFORM,
                                                 mixing=arche.MIX_FIXED, w_fixed=0.9))
    c = ctx.solve(w.pos)
    assert abs(c["F"] - r.th.F) <= 1e-11 * abs(r.th.F)
    ctx.close()


def test_error_paths(small_solved):
    w, r = small_solved["rand4_16c_10eV"]
    ctx = arche.Context.from_workload(w, opts_of(w, scf_max_iter=2, init=arche.INIT_UNIFORM))
    with pytest.raises(arche.ArcheError) as e:
        ctx.forces()
    assert e.value.status == arche.ESTATE
    res = ctx.solve(w.pos, allow_noconv=True)
    assert not res["converged"] and res["scf_iters"] == 2 and math.isfinite(res["F"])
    with pytest.raises(arche.ArcheError) as e:
        ctx.solve(w.pos)
    assert e.value.status == arche.ENOCONV
    bad = w.pos.copy()
    bad[1, 2] = np.nan
    with pytest.raises(arche.ArcheError) as e:
        ctx.solve(bad)
    assert e.value.status == arche.EINVAL
    ctx.close()


def oracle_at_gpu_state(w, ctx, res, atoms=None, forces=True):
    """Oracle evaluation of F, P and forces at the GPU's converged (n_a, eta)."""
    s = system_of(w)
    ion = oscf.ionic_setup(s)
    Vi = ctx.debug("Vi")
    eta = (res["mu"] - Vi) / w.kT
    n = ctx.density()
    sr = oscf.SCFResult(n, eta, res["mu"], Vi, res["scf_iters"], res["residual"], True)
    return s, ion, n, oth.evaluate(s, ion, sr, forces=forces, atoms=atoms)


def fixed_point_residual(s, ion, n):
    V, _ = oscf.effective_potential(s, ion, n)
    mu, _ = oscf.solve_mu(s, V)
    n2 = ofd.density((mu - V) / s.kT, s.kT)
    return float(np.sqrt(np.sum((n2 - n) ** 2) / np.sum(n * n))), mu


@pytest.mark.parametrize("wname", ["fcc32", "fcc256"])
def test_full_size_config(wname):
    w = getattr(W, wname)()
    say("full-size", w.name)
    ctx = arche.Context.from_workload(w, opts_of(w, init=arche.INIT_UNIFORM))
    res = ctx.solve(w.pos)
    assert res["converged"]
    Fg = ctx.forces()
    s, ion, n, th = oracle_at_gpu_state(w, ctx, res)
    assert abs(res["F"] - th.F) <= 1e-11 * abs(th.F)
    assert abs(res["P"] - th.P) <= 1e-10 * abs(th.P)
    assert force_err(Fg, th.forces) <= RTOL
    rfp, mu = fixed_point_residual(s, ion, n)
    assert rfp <= 100 * 1e-10, rfp
    assert abs(mu - res["mu"]) <= 1e-8 * max(abs(mu), w.kT)
    assert abs(s.grid.integrate(n) - s.Ne) <= 1e-12 * s.Ne
    ctx.close()


def test_rand1024_sampled():
    w = W.rand1024()
    say("full-size", w.name)
    ctx = arche.Context.from_workload(w, opts_of(w, init=arche.INIT_UNIFORM))
    res = ctx.solve(w.pos)
    assert res["converged"]
    Fg = ctx.forces()
    atoms = [0, 1, 511, 1023]
    s, ion, n, th = oracle_at_gpu_state(w, ctx, res, atoms=atoms)
    assert abs(res["F"] - th.F) <= 1e-11 * abs(th.F)
    assert abs(res["P"] - th.P) <= 1e-10 * abs(th.P)
    assert force_err(Fg[atoms], th.forces) <= RTOL
    rfp, mu = fixed_point_residual(s, ion, n)
    assert rfp <= 100 * 1e-10, rfp
    ctx.close()


def test_plane_grid_iteration_parity():
    """Iteration-by-iteration parity on a grid with N_y = N_z = 128, the shape on
    which the SCF iteration runs the plane FFT passes (z and y in one pass, with
    the square root, the mixing and the U_vW sums fused into them) and the paired
    launches: 128 atoms in a 16 x 128 x 128 slab (0.3-0.4 bohr spacing), seven
    iterations from the uniform density with More's weight on from the third
    (trust bound lifted, so U_H, U_xc, U_vW and K all enter), against the
    oracle's SCF loop (Sec. 2.5, 2.5.2): every residual and every weight."""
    w = W.small_random(128, 64, 2.7, 10.0, seed=21, shape=(16, 128, 128), stretch=(0.2, 2.2361, 2.2361))
    say("plane-grid iterations", w.name)
    its = 7
    ctx = arche.Context.from_workload(w, opts_of(w, init=arche.INIT_UNIFORM, scf_tol=1e-300, scf_max_iter=its,
                                                 more_warmup=2, more_trust=1e30))
    ctx.solve(w.pos, allow_noconv=True)
    h = ctx.history()
    ctx.close()
    assert h.shape[0] == its
    s = system_of(w)
    ion = oscf.ionic_setup(s)
    n0 = np.full(s.shape, s.Ne / s.grid.volume)
    say("oracle iterations")
    r = oscf.scf(s, ion, n0, mixing="more", tol=1e-300, max_iter=its, warmup=2, w_fixed=w.w_fixed, more_trust=1e30)
    say("residuals gpu", h[:, 1], "oracle", r.history)
    say("weights gpu", h[:, 2], "oracle", r.weights)
    for t in range(its):
        assert abs(h[t, 1] - r.history[t]) <= 1e-9 * r.history[t], (t, h[t, 1], r.history[t])
    # the last iteration raises done before its weight is formed on the GPU
    for t in range(its - 1):
        assert abs(h[t, 2] - r.weights[t]) <= 1e-9, (t, h[t, 2], r.weights[t])
    # More's own weight (not a clamp) was taken in some iterations
    assert any(abs(x - round(x / 0.05) * 0.05) > 1e-6 for x in r.weights[2:its - 1])


def test_cubic_128_iteration_parity():
    """Iteration-by-iteration parity on a 128^3 grid, the shape on which the
    iteration also takes the Laplacian's x round trip (MODE 4: forward x pass,
    multiply, inverse x pass on one tile), runs the Hartree C2R's x pass in one
    launch with R2C(sqrt n_o)'s plane pass and pairs the two C2R plane passes
    (-> V_H, -> lap sqrt(n_o)): 128 atoms, five iterations from the uniform
    density with More's weight on from the third (trust bound lifted), against
    the oracle's SCF loop (Sec. 2.5, 2.5.2): every residual and weight, and
    element by element the last iteration's potential V_i (Sec. 2.2, built on
    V_H and lap sqrt(n_i) from the previous iteration's passes) and active
    density n_a."""
    w = W.small_random(128, 128, 2.7, 10.0, seed=31)
    say("128^3 iterations", w.name)
    its = 5
    ctx = arche.Context.from_workload(w, opts_of(w, init=arche.INIT_UNIFORM, scf_tol=1e-300, scf_max_iter=its,
                                                 more_warmup=2, more_trust=1e30))
    ctx.solve(w.pos, allow_noconv=True)
    h = ctx.history()
    Vi = ctx.debug("Vi")
    na = ctx.debug("n_a")
    ctx.close()
    assert h.shape[0] == its
    s = system_of(w)
    ion = oscf.ionic_setup(s)
    n0 = np.full(s.shape, s.Ne / s.grid.volume)
    say("oracle iterations")
    r = oscf.scf(s, ion, n0, mixing="more", tol=1e-300, max_iter=its, warmup=2, w_fixed=w.w_fixed, more_trust=1e30)
    say("residuals gpu", h[:, 1], "oracle", r.history)
    say("weights gpu", h[:, 2], "oracle", r.weights)
    for t in range(its):
        assert abs(h[t, 1] - r.history[t]) <= 1e-9 * r.history[t], (t, h[t, 1], r.history[t])
    for t in range(its - 1):
        assert abs(h[t, 2] - r.weights[t]) <= 1e-9, (t, h[t, 2], r.weights[t])
    assert any(abs(x - round(x / 0.05) * 0.05) > 1e-6 for x in r.weights[2:its - 1])
    dv = np.max(np.abs(Vi - r.V)) / np.max(np.abs(r.V))
    dn = np.max(np.abs(na - r.n) / r.n)
    say("max |V_i - V| / max |V|", dv, "max |n_a - n| / n", dn)
    assert dv <= 1e-9 and dn <= 1e-9


def test_plain_and_cooperative_launch_agree():
    """With exclusive_device set, the SCF kernel runs as a plain launch while its
    context is the only one alive and as a cooperative launch otherwise (the
    default is always cooperative); the arithmetic is the same, so the two
    solves are bit-identical (density, F, iterations)."""
    import gc
    gc.collect()
    L = arche.load()
    w = W.small_random(8, 20, 2.7, 5.0, seed=12)
    ctx = arche.Context.from_workload(w, opts_of(w, init=arche.INIT_UNIFORM, exclusive_device=1))
    assert L.arche_debug_live_contexts() == 1, "another context is still alive"
    r1 = ctx.solve(w.pos)
    n1 = ctx.density()
    other = arche.Context.from_workload(w, opts_of(w, init=arche.INIT_UNIFORM, exclusive_device=1))
    assert L.arche_debug_live_contexts() == 2
    r2 = ctx.solve(w.pos)
    n2 = ctx.density()
    other.close()
    ctx.close()
    assert r1["converged"] and r2["converged"]
    assert r1["scf_iters"] == r2["scf_iters"]
    assert r1["F"] == r2["F"] and r1["mu"] == r2["mu"]
    assert np.array_equal(n1, n2)
