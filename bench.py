#!/usr/bin/env python
"""Benchmark of the FP64 orbital-free MD step on one MI355X.

Workload (default): 1024 Al atoms at 2.7 g/cm^3, T = 10 eV, 128^3 grid,
Thomas-Fermi + 0.2 von Weizsaecker + LDA, empty-core pseudopotential
(r_c = 1.1 bohr), SCF tolerance 1e-10, 0.2 fs Verlet steps with the
one-center initial density and More mixing.  Inputs are seeded synthetic
positions and Maxwell-Boltzmann velocities.

A step is one MD step: structure factor and ionic field, one-center guess,
the SCF to convergence, free energy and pressure, forces, Verlet update.
Prints one JSON line.  The value is SCF iterations per second over the timed
steps; the wall time per MD step is ms_per_step.  More comparisons ride along
(untimed for `value`): "batch" (64 independent 108-atom snapshots solved one
after another vs in one batch), "learned_init" and "learned_init_128" (plain
guess vs previous density vs the learned proposal on 256-atom MD at 64^3 and on
the benchmark's own 1024-atom cell at 128^3), "ablation" (the setups of the
paper's SCF-count comparison) and "large_snapshot" (4000 atoms at 192^3).

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--batch N] [--learned K]
                  [--ablation K] [--large 0|1] [--no-cpu-baseline] [--copy-probe MIB]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6  # vector FP64: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
# the timed steps time one SCF-kernel launch in this many with a HIP event pair
PROF_SAMPLE = 16
# algorithmic FP64 flops per grid point of the SCF kernel: each evaluation of
# N(mu) (I_{1/2} with its derivatives and the sums) ~130, the potential
# assembly with LDA xc ~60; the kernel makes m evaluations (the one at the
# previous mu during the assembly, then Newton's, the last of which forms the
# active density)
FLOP_PER_FD_PASS = 130.0
FLOP_ASSEMBLY_XC = 60.0
# algorithmic HBM bytes per grid point of one whole SCF iteration (every pass
# at its one-read-one-write minimum, von Weizsaecker and More mixing included)
ITER_BYTES_PER_POINT = 216.0
METRIC = "SCF iters/s + wall s per MD step (plain vs learned-init/batched), 1024 Al, 128³"


def kernel_bytes(name, ng, nh, newton_per_launch, more_frac=0.0):
    """Algorithmic HBM bytes of one launch of each timed kernel class."""
    if name == "scf_active":
        # potential assembly: read n_i, V^ie, V_H, lap sqrt(n_i) (32 B/pt); the Newton
        # passes read nothing (V_i and v_xc(n_i) stay in LDS); the last phase reads n_i and
        # writes n_a (16 B/pt); V_i is written only by the iteration that ends the solve.
        # Once More's weight is on (a fraction more_frac of the launches) the last phase
        # also reads lap sqrt(n_i) and writes (n_i - n_a)/sqrt(n_a) for the U_vW pass
        return ng * (48.0 + 16.0 * more_frac)
    if name == "fft_z":
        # the z pass, or on N_y = N_z grids the fused z+y plane pass: real field in/out +
        # half spectrum out/in
        return ng * 8.0 + nh * 16.0
    if name == "fft_strided":
        return 2.0 * nh * 16.0  # half spectrum read and written in place
    raise KeyError(name)


def sources_sha256(paths):
    """SHA-256 of the kernel's source files, in order."""
    h = hashlib.sha256()
    for p in paths:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()


def counter_record(kind, name):
    """A committed rocprofv3 counter record (profiles/<kind>_<name>.json), or None
    when absent or taken before the kernel's sources last changed."""
    path = os.path.join(ROOT, "profiles", "%s_%s.json" % (kind, name))
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        if sources_sha256(d["sources"]) != d["sources_sha256"]:
            return None
        return d
    except Exception:
        return None


def counter_flops_for(name):
    """FP64 flops per launch from the committed rocprofv3 counter run
    (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes), or None when absent or stale."""
    d = counter_record("flops", name)
    return None if d is None else float(d["fp64_flops_per_launch"])


def traffic_for(name):
    """HBM bytes per launch from committed rocprofv3 counter runs (FETCH_SIZE and
    WRITE_SIZE, scaled by a copy of known size), or None when absent or stale."""
    d = counter_record("traffic", name)
    return None if d is None else float(d["bytes_per_launch"])


def cpu_baseline(w, seconds):
    """The oracle on the host cores: SCF iterations/s on the same workload, over a
    bounded sample of iterations from the uniform start."""
    import numpy as np
    from oracle import scf as oscf

    s = oscf.System(w.cell, w.grid, w.pos, w.species, w.Z, w.rc, w.mass, w.kT, w.lam, w.xc)
    t0 = time.perf_counter()
    ion = oscf.ionic_setup(s)
    n0, _ = oscf.initial_density(s, ion)
    setup = time.perf_counter() - t0
    iters = 0
    t0 = time.perf_counter()
    n = n0
    mu = None
    while True:
        r = oscf.scf(s, ion, n, mixing="more", tol=0.0, max_iter=1, w_fixed=w.w_fixed, mu0=mu)
        iters += 1
        mu = r.mu
        n = r.n + r.weights[-1] * (n - r.n) if r.weights else r.n
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": iters / dt, "unit": "SCF iters/s", "cores": cores, "kind": "oracle",
            "sample": "%d oracle SCF iterations of %s from the uniform start (%.1f s; structure factor "
                      "and ionic field setup %.1f s not counted)" % (iters, w.name, dt, setup)}


def bench_batch(count):
    """The batched-solve workload: `count` independent 108-atom snapshots (48^3-72^3
    grids, 1.5-5.4 g/cm^3, 1-20 eV), one SCF each from the uniform density.  Times
    the snapshots solved one after another on their own contexts against the same
    snapshots in one batch (first solve, which includes the autotuner's timing
    rounds, and a second solve with the tuned schedule), and checks that the
    batched results are bit-identical to the sequential ones."""
    import numpy as np
    import torch

    from paper_2606_13283_amd import arche
    from paper_2606_13283_amd import workloads as W

    ws = W.batch64(count)

    def opts(w):
        return arche.Options(w_fixed=w.w_fixed, lambda_vw=w.lam, xc=arche.XC_LDA if w.xc else arche.XC_NONE,
                             init=arche.INIT_UNIFORM, scf_tol=1e-10)

    # one after another, each on its own context with no other context alive (the
    # single-system path at its fastest: plain launches of the SCF kernel); the
    # clock covers the solves, not the contexts' creation
    seq = []
    t_seq = 0.0
    for w in ws:
        o = opts(w)
        o.exclusive_device = 1
        c = arche.Context.from_workload(w, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        seq.append(c.solve(w.pos))
        t_seq += time.perf_counter() - t0
        c.close()
    print("[bench] batch: %d sequential solves in %.3f s (%d SCF iterations)" % (
        len(ws), t_seq, sum(r["scf_iters"] for r in seq)), file=sys.stderr, flush=True)
    b = arche.Batch.from_workloads(ws, opts)
    t0 = time.perf_counter()
    r1 = b.solve([w.pos for w in ws])
    t_b1 = time.perf_counter() - t0
    info1 = b.info()
    t0 = time.perf_counter()
    r2 = b.solve([w.pos for w in ws])
    t_b2 = time.perf_counter() - t0
    info2 = b.info()
    b.close()
    print("[bench] batch: batched %.3f s (tuning solve %.3f s)" % (t_b2, t_b1), file=sys.stderr, flush=True)
    same = all(x["F"] == y["F"] and x["P"] == y["P"] and x["scf_iters"] == y["scf_iters"]
               for x, y in zip(seq, r2))
    iters = sum(r["scf_iters"] for r in seq)
    grids = sorted({w.grid[0] for w in ws})
    return {"workload": "batch%d_108Al" % len(ws), "snapshots": len(ws), "grids": grids,
            "scf_iters_total": iters, "sequential_s": t_seq, "batched_s": t_b2, "batched_first_s": t_b1,
            "speedup": t_seq / t_b2, "snapshots_per_s": len(ws) / t_b2,
            "scf_iters_per_s_sequential": iters / t_seq, "scf_iters_per_s_batched": iters / t_b2,
            "bit_identical_to_sequential": bool(same), "schedule": info2, "tuning": info1}


def bench_learned(steps_train, epochs, steps_eval, size=64):
    """The learned initial density.  size 64: 256 Al atoms at 64^3, training
    samples from plain MD at 2, 4, 6, 8, 10 eV (`steps_train` steps each), a
    held-out 5 eV trajectory.  size 128: the 1024-atom, 128^3, 10 eV cell,
    samples from three other seeded cells (`steps_train` steps each), the
    benchmark's own trajectory held out.  `epochs` of Adam on the GPU, then
    `steps_eval` MD steps solved from the plain guess, from the previous
    converged density alone and from the learned proposal at the same positions.
    Wall time per MD step and SCF iterations of each, the free energies
    agreeing to 1e-9."""
    import numpy as np
    import torch

    from paper_2606_13283_amd import arche
    from paper_2606_13283_amd import learned as LN
    from paper_2606_13283_amd import workloads as W

    if size == 64:
        ws = [W.fcc256_at(T, seed=100 + i) for i, T in enumerate((2.0, 4.0, 6.0, 8.0, 10.0))]
        w = W.fcc256_at(5.0, seed=300)
        desc = "fcc256_64^3 MD at 5 eV (held out), trained on 2-10 eV"
    else:
        ws = [W.rand1024(seed=101 + i) for i in range(3)]
        w = W.rand1024()
        desc = "rand1024_128^3_10eV MD (the benchmark's trajectory, held out), trained on three other seeded cells"
    t0 = time.perf_counter()
    samples = LN.generate(ws, steps=steps_train)
    t_gen = time.perf_counter() - t0
    net = arche.Net(w.grid)
    net.set_params(LN.init_params(0))
    data = [s for s, _ in samples]
    n0s = [LN.n0_of(ws[0])] * len(data)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = LN.train(net, data, n0s, epochs=epochs, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_train_steps = epochs * len(data)
    # one variant at a time, each with only its own context alive, at the positions
    # of the plain trajectory (several live contexts make one of them run slower)
    kinds = {"plain": arche.INIT_ONE_CENTER, "previous_density": arche.INIT_KEEP, "learned": arche.INIT_LEARNED}
    wall = {k: 0.0 for k in kinds}
    iters = {k: [] for k in kinds}
    Fs = {k: [] for k in kinds}
    positions = None
    for k, init in kinds.items():
        tr = LN.Trajectory(w, init=init, net=net if k == "learned" else None)
        if positions is None:
            positions = []
        for step in range(steps_eval):
            if k == "previous_density":
                tr.ctx.set_density(tr.ctx.density())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if k == "plain":
                res, _ = tr.step()
                positions.append(tr.pos.copy())
            else:
                res = tr.solve_at(positions[step])
            torch.cuda.synchronize()
            wall[k] += time.perf_counter() - t0
            iters[k].append(res["scf_iters"])
            Fs[k].append(res["F"])
        tr.close()
    net.close()
    same = all(abs(a - b) <= 1e-9 * abs(a) for k in ("previous_density", "learned") for a, b in zip(Fs["plain"], Fs[k]))
    print("[bench] learned %d^3: iterations plain %.1f, previous density %.1f, learned %.1f" % ((size,) + tuple(
        float(np.mean(iters[k])) for k in ("plain", "previous_density", "learned"))), file=sys.stderr, flush=True)
    return {"workload": desc, "samples": len(data),
            "epochs": epochs, "sample_generation_s": t_gen, "training_s": t_train,
            "training_steps_per_s": n_train_steps / t_train, "loss_first_last_epoch": [hist[0], hist[-1]],
            "md_steps": steps_eval,
            "wall_s_per_md_step": {k: wall[k] / steps_eval for k in wall},
            "scf_iters_per_md_step": {k: float(np.mean(iters[k])) for k in iters},
            "wall_reduction_vs_plain": {k: 1.0 - wall[k] / wall["plain"] for k in ("previous_density", "learned")},
            "scf_iters_each_step": iters, "free_energy_agrees_1e-9": bool(same)}


def bench_ablation(steps):
    """The SCF-count ablation of Sec. 2.5.3 (Fig. convergence) on the 256-atom fcc
    cell at 64^3 and 5 eV: MD steps with (A) the uniform initial density and
    fixed mixing, (B) uniform and More's weight, (C) the one-center guess and
    fixed mixing, (D) both.  Positions follow setup D's trajectory; every setup
    solves at the same positions.  Total SCF iterations per setup, and the
    largest relative spread of the free energy across setups at each step."""
    import numpy as np

    from paper_2606_13283_amd import arche
    from paper_2606_13283_amd import workloads as W

    w = W.fcc256()
    setups = {"A": (arche.INIT_UNIFORM, arche.MIX_FIXED), "B": (arche.INIT_UNIFORM, arche.MIX_MORE),
              "C": (arche.INIT_ONE_CENTER, arche.MIX_FIXED), "D": (arche.INIT_ONE_CENTER, arche.MIX_MORE),
              # B with More's weight exactly as printed (Hartree-only U, second-order K)
              "B_printed": (arche.INIT_UNIFORM, arche.MIX_MORE_PRINTED)}
    ctx = {}
    for k, (init, mix) in setups.items():
        o = arche.Options(w_fixed=w.w_fixed, lambda_vw=w.lam, xc=arche.XC_LDA, init=init, mixing=mix,
                          scf_tol=1e-10, scf_max_iter=20000)
        ctx[k] = arche.Context.from_workload(w, o)
    m = np.array([w.mass[s] for s in w.species])[:, None]
    r = w.pos.copy()
    iters = {k: [] for k in setups}
    fallback = {k: [] for k in setups}
    spread = []
    t0 = time.perf_counter()
    res = {k: c.solve(r, allow_noconv=True) for k, c in ctx.items()}
    F = ctx["D"].forces()
    r_prev = r - w.vel * w.dt + F * w.dt ** 2 / (2 * m)
    for step in range(steps):
        r_next = 2 * r - r_prev + F * w.dt ** 2 / m
        res = {k: c.solve(r_next, allow_noconv=True) for k, c in ctx.items()}
        for k in setups:
            iters[k].append(res[k]["scf_iters"] if res[k]["converged"] else None)
            fallback[k].append(int(res[k]["used_fallback"]))
        Fs = [res[k]["F"] for k in setups if res[k]["converged"]]
        spread.append((max(Fs) - min(Fs)) / abs(res["D"]["F"]))
        F = ctx["D"].forces()
        r_prev, r = r, r_next
        print("[bench] ablation step %d: %s" % (step, {k: iters[k][-1] for k in setups}), file=sys.stderr, flush=True)
    for c in ctx.values():
        c.close()
    return {"workload": w.name, "md_steps": steps, "scf_tol": 1e-10,
            "total_scf_iters": {k: (int(sum(v)) if None not in v else None) for k, v in iters.items()},
            "not_converged_steps": {k: sum(x is None for x in v) for k, v in iters.items()},
            "scf_iters_each_step": iters, "one_center_fallback_each_step": {"C": fallback["C"], "D": fallback["D"]},
            "max_rel_F_spread": max(spread) if spread else None, "seconds": time.perf_counter() - t0}


def bench_large(w_name="rand4000"):
    """The 4000-atom cell at 192^3 and 10 eV: one SCF from the uniform density
    (then one more, timed), forces and stress; SCF iterations/s and grid-point
    updates/s of the single-snapshot solve at the largest configured grid."""
    import torch

    from paper_2606_13283_amd import arche
    from paper_2606_13283_amd import workloads as W

    w = getattr(W, w_name)()
    o = arche.Options(w_fixed=w.w_fixed, init=arche.INIT_UNIFORM, scf_tol=1e-10, exclusive_device=1)
    ctx = arche.Context.from_workload(w, o)
    r0 = ctx.solve(w.pos)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.solve(w.pos)
    t_solve = time.perf_counter() - t0
    t0 = time.perf_counter()
    ctx.forces()
    t_forces = time.perf_counter() - t0
    t0 = time.perf_counter()
    ctx.stress()
    t_stress = time.perf_counter() - t0
    ctx.close()
    ng = w.grid[0] * w.grid[1] * w.grid[2]
    print("[bench] large: %s %d SCF iterations in %.3f s" % (w.name, r["scf_iters"], t_solve), file=sys.stderr,
          flush=True)
    return {"workload": w.name, "n_atoms": int(w.pos.shape[0]), "grid": list(w.grid), "scf_iters": r["scf_iters"],
            "solve_s": t_solve, "scf_iters_per_s": r["scf_iters"] / t_solve,
            "grid_point_updates_per_s": ng * r["scf_iters"] / t_solve, "forces_s": t_forces, "stress_s": t_stress,
            "F": r["F"], "P": r["P"], "first_solve_same_F": r0["F"] == r["F"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rand1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--batch", type=int, default=64, help="snapshots of the batched-solve comparison (0: skip)")
    ap.add_argument("--learned", type=int, default=8, help="MD steps of the learned-init comparison (0: skip)")
    ap.add_argument("--large", type=int, default=1, help="1: time one SCF of the 4000-atom 192^3 cell (0: skip)")
    ap.add_argument("--ablation", type=int, default=6,
                    help="MD steps of the A/B/C/D SCF-count ablation on the 256-atom cell (0: skip)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device 5 times (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the whole path on a single MI355X "
              "(sharding over several GPUs is described, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_13283_amd import arche
    from paper_2606_13283_amd import workloads as W

    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 5}))
        return
    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    arche.load()
    w = getattr(W, args.workload)()
    stream = torch.cuda.current_stream().cuda_stream
    # the benchmark owns the GPU: the SCF kernel may be a plain launch
    opts = arche.Options(w_fixed=w.w_fixed, init=arche.INIT_ONE_CENTER, scf_tol=1e-10, exclusive_device=1)
    ctx = arche.Context.from_workload(w, opts, stream=stream)
    pos = w.pos.copy()
    vel = w.vel.copy() if w.vel is not None else np.zeros_like(pos)
    dt = w.dt
    ng = w.grid[0] * w.grid[1] * w.grid[2]
    nh = w.grid[0] * w.grid[1] * (w.grid[2] // 2 + 1)
    L = arche.load()
    tiles = {"y": int(L.arche_fft_tile(0, w.grid[1], -1)), "x": int(L.arche_fft_tile(1, w.grid[0], -1)),
             "z": int(L.arche_fft_tile(2, w.grid[2], -1))}

    t0 = time.perf_counter()
    first = ctx.solve(pos)
    first_s = time.perf_counter() - t0
    print("[bench] first solve: %d SCF iterations in %.3f s" % (first["scf_iters"], first_s), file=sys.stderr,
          flush=True)
    F_prev = first["F"]
    for k in range(args.warmup):
        pos, vel, F, res = ctx.md_step(dt, pos, vel)
        F_prev = res["F"]
        print("[bench] warmup step %d: %d SCF iterations" % (k, res["scf_iters"]), file=sys.stderr, flush=True)
    mass = np.array([w.mass[s] for s in w.species])[:, None]

    # the timed steps time the SCF kernel alone, one launch in PROF_SAMPLE
    # (every timed launch adds an event pair and ~10 us of idle GPU before the
    # next launch; sampling keeps that out of the other launches)
    ctx.profile(True, kinds=("scf_active",))
    ctx.profile_sample(PROF_SAMPLE)
    ctx.profile_reset()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    t0 = time.perf_counter()
    iters = newton = more_iters = 0
    per_step, fallback, Ki, conserved = [], [], [], []
    for k in range(args.steps):
        pos, vel, F, res = ctx.md_step(dt, pos, vel)
        iters += res["scf_iters"]
        newton += res["newton_iters"]
        per_step.append(res["scf_iters"])
        more_iters += int(np.sum(ctx.history()[:, 8] != 0))
        fallback.append(int(res["used_fallback"]))
        # the step returns v(t) (central difference) and F at t + dt: pair v(t) with
        # the previous step's free energy F(t) for the conserved K^i + F
        kin = 0.5 * float(np.sum(mass * vel * vel))
        Ki.append(kin)
        conserved.append(kin + F_prev)
        F_prev = res["F"]
        print("[bench] step %d: %d SCF iterations, F = %.12f Ha, P = %.6e Ha/bohr^3" % (
            k, res["scf_iters"], res["F"], res["P"]), file=sys.stderr, flush=True)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_s = ev0.elapsed_time(ev1) / 1e3
    prof = ctx.profile_read()
    # one more MD step, untimed, with every kernel class timed, for the table
    ctx.profile(True)
    ctx.profile_reset()
    pos, vel, F, res = ctx.md_step(dt, pos, vel)
    prof_all = ctx.profile_read()
    ctx.close()

    newton_per_launch = newton / max(iters, 1)
    more_frac = more_iters / max(iters, 1)

    def table(pr, nl):
        out = {}
        for name, (ms, n) in pr.items():
            if n:
                b = kernel_bytes(name, ng, nh, nl, more_frac)
                out[name] = {"total_ms": ms, "launches": n, "avg_us": 1e3 * ms / n,
                             "alg_bytes_per_launch": b, "GBps": b / (ms / n * 1e-3) / 1e9}
        return out

    # dominant kernel: the SCF kernel (one launch per iteration, the largest
    # share of the iteration); measured over the timed steps
    kernels = table(prof, newton_per_launch)
    kernels_step = table(prof_all, res["newton_iters"] / max(res["scf_iters"], 1))
    dom = "scf_active"
    d = kernels[dom]
    traffic = traffic_for(dom)
    # the SCF kernel is bound by FP64 arithmetic (Fermi-Dirac evaluations), not
    # HBM: price it against the FP64 vector peak with its algorithmic flops
    flops = ng * (FLOP_PER_FD_PASS * newton_per_launch + FLOP_ASSEMBLY_XC)
    tflops = flops / (d["avg_us"] * 1e-6) / 1e12
    roofline = {"bound": "alu", "kernel": dom, "achieved": tflops, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": tflops / PEAK_FP64_TFLOPS, "traffic": traffic,
                "alg_flops_per_launch": flops, "mu_evaluations_per_launch": newton_per_launch,
                "more_weight_on_fraction": more_frac,
                "counter_fp64_flops_per_launch": counter_flops_for(dom),
                "alg_bytes_per_launch": d["alg_bytes_per_launch"], "hbm_GBps": d["GBps"],
                "hbm_frac": d["GBps"] / PEAK_HBM_GBS, "avg_launch_us": d["avg_us"]}
    # the whole iteration against HBM: kernel time per iteration of the timed
    # classes (one untimed step with every class bracketed)
    n_it = max(res["scf_iters"], 1)
    cls = {k: {"us_per_iter": 1e3 * v["total_ms"] / n_it, "launches_per_iter": v["launches"] / n_it}
           for k, v in kernels_step.items()}
    it_us = sum(v["us_per_iter"] for v in cls.values())
    iteration = {"kernel_us_per_iter": it_us, "alg_bytes_per_iter": ITER_BYTES_PER_POINT * ng,
                 "hbm_GBps": ITER_BYTES_PER_POINT * ng / (it_us * 1e-6) / 1e9,
                 "hbm_frac": ITER_BYTES_PER_POINT * ng / (it_us * 1e-6) / 1e9 / PEAK_HBM_GBS,
                 "wall_us_per_iter": 1e6 * wall / max(iters, 1), "classes": cls}
    value = iters / wall
    out = {
        "metric": METRIC, "value": value, "unit": "SCF iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "n_atoms": int(pos.shape[0]), "grid": list(w.grid),
                   "T_eV": w.kT * W.HARTREE_EV, "dt_fs": 0.2, "scf_tol": 1e-10, "init": "one-center",
                   "mixing": "More", "functional": "TF+0.2vW+LDA"},
        "wall_s_per_md_step": wall / args.steps,
        "scf_iters_per_md_step": iters / args.steps,
        "grid_point_updates_per_s": ng * value,
        "event_s": ev_s,
        "scf_iters_each_step": per_step,
        "used_fallback_each_step": fallback,
        "ion_kinetic_each_step": Ki,
        "conserved_Ki_plus_F_each_step": conserved,
        "conserved_drift_rel": (conserved[-1] - conserved[0]) / abs(conserved[0]) if conserved else None,
        "first_solve": {"scf_iters": first["scf_iters"], "s": first_s},
        "kernels": kernels,
        "kernels_timed_one_launch_in": PROF_SAMPLE,
        "kernels_all_classes_one_untimed_step": kernels_step,
        "roofline": roofline,
        "iteration_roofline": iteration,
        "fft_tile_variants": tiles,
    }
    if args.batch > 0:
        out["batch"] = bench_batch(args.batch)
    if args.learned > 0:
        out["learned_init"] = bench_learned(16, 12, args.learned)
        out["learned_init_128"] = bench_learned(6, 6, min(args.learned, 4), size=128)
    if args.ablation > 0:
        out["ablation"] = bench_ablation(args.ablation)
    if args.large > 0:
        out["large_snapshot"] = bench_large()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
