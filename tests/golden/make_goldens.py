"""Writes the stored expected values of the full-size parity tests.

Every value here comes from the FP64 CPU oracle (`oracle/`) solving the seeded
workload itself; nothing is read from the HIP path.  The inputs come from the
seeded input generators (`paper_2606_13283_amd/workloads.py`, which holds none
of the method's arithmetic).

    python tests/golden/make_goldens.py fcc256 rand1024 rand4000 fcc256_md

Each name writes tests/golden/oracle_<name>.json:
  static workloads: one SCF from the uniform density (Sec. 2.5) to a relative
    residual of 1e-12, then F, E, P and every term (Sec. 2.6), mu, forces
    (eq. force; all atoms, or a seeded sample of atoms on the largest cell),
    and the converged density at a seeded sample of grid points;
  fcc256_md: the 256-atom fcc cell's Verlet trajectory (Sec. 2.1) for three
    steps after the initial solve, each step started from the one-center guess
    (Sec. 2.5.1) of the previous step: positions, velocities, F, P, mu and all
    forces per step.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import md as omd  # noqa: E402
from oracle import scf as oscf  # noqa: E402
from paper_2606_13283_amd import workloads as W  # noqa: E402

TOL = 1e-12
DENSITY_SAMPLES = 512
FORCE_SAMPLE_ATOMS = 64  # atoms whose forces are stored when the cell has more than 1024


def system_of(w):
    return oscf.System(w.cell, w.grid, w.pos, w.species, w.Z, w.rc, w.mass, w.kT, w.lam, w.xc)


def thermo_dict(th):
    return dict(F=th.F, E=th.E, P=th.P, terms={k: float(v) for k, v in th.terms.items()},
                P_terms={k: float(v) for k, v in th.P_terms.items()})


def sample_points(shape, seed):
    rng = np.random.default_rng(seed)
    ng = int(np.prod(shape))
    idx = np.sort(rng.choice(ng, size=min(DENSITY_SAMPLES, ng), replace=False))
    return idx


def static(name):
    w = getattr(W, name)()
    s = system_of(w)
    n_atoms = s.pos.shape[0]
    atoms = None
    if n_atoms > 1024:
        atoms = sorted(int(a) for a in np.random.default_rng(7).choice(n_atoms, FORCE_SAMPLE_ATOMS, replace=False))
    t0 = time.time()
    ion = oscf.ionic_setup(s)
    t_ion = time.time() - t0
    n0, _ = oscf.initial_density(s, ion, "uniform")
    t0 = time.time()
    res = oscf.scf(s, ion, n0, mixing="more", tol=TOL, w_fixed=w.w_fixed, max_iter=5000)
    t_scf = time.time() - t0
    assert res.converged, name
    from oracle import thermo
    th = thermo.evaluate(s, ion, res, forces=True, atoms=atoms)
    idx = sample_points(s.shape, 11)
    out = dict(workload=w.name, grid=list(w.grid), cell=list(w.cell), scf_tol=TOL, init="uniform",
               w_fixed=w.w_fixed, scf_iters=res.iters, residual=res.residual, mu=res.mu,
               **thermo_dict(th),
               force_atoms=list(range(n_atoms)) if atoms is None else atoms,
               forces=th.forces.tolist(),
               density_index=idx.tolist(), density=res.n.reshape(-1)[idx].tolist(),
               oracle_seconds=dict(ionic_setup=t_ion, scf=t_scf))
    return out


def fcc256_md(steps=3):
    w = W.fcc256()
    s = system_of(w)
    m = omd.masses(s)
    dt = w.dt
    r0 = omd.solve_at(s, init="uniform", tol=TOL)
    assert r0.scf.converged
    out = dict(workload=w.name, grid=list(w.grid), cell=list(w.cell), scf_tol=TOL, dt=dt,
               init="one_center", w_fixed=w.w_fixed, start=dict(pos=s.pos.tolist(), vel=w.vel.tolist(),
                                                                F=r0.th.F, P=r0.th.P, mu=r0.scf.mu,
                                                                forces=r0.th.forces.tolist(),
                                                                scf_iters=r0.scf.iters),
               steps=[])
    r_prev = omd.verlet_start(s.pos, w.vel, r0.th.forces, m, dt)
    r_cur, F_cur, prev = s.pos, r0.th.forces, r0
    for step in range(steps):
        r_next, v = omd.verlet_step(r_cur, r_prev, F_cur, m, dt)
        s_next = s.with_positions(r_next)
        cur = omd.solve_at(s_next, init="one_center", prev=(prev.nhat, prev.ion.SZ), tol=TOL,
                           max_iter=5000)
        assert cur.scf.converged, step
        out["steps"].append(dict(pos=r_next.tolist(), vel=v.tolist(), F=cur.th.F, E=cur.th.E, P=cur.th.P,
                                 mu=cur.scf.mu, forces=cur.th.forces.tolist(), scf_iters=cur.scf.iters,
                                 used_fallback=bool(cur.scf.used_fallback)))
        print("fcc256_md step %d: %d iterations, fallback %s, F %.15g" % (
            step, cur.scf.iters, cur.scf.used_fallback, cur.th.F), flush=True)
        r_prev, r_cur, F_cur, prev = r_cur, r_next, cur.th.forces, cur
    return out


def main(names):
    for name in names:
        t0 = time.time()
        out = fcc256_md() if name == "fcc256_md" else static(name)
        path = os.path.join(HERE, "oracle_%s.json" % name)
        with open(path, "w") as f:
            json.dump(out, f, indent=0)
        print("%s: written in %.0f s" % (path, time.time() - t0), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["fcc256", "rand1024", "rand4000", "fcc256_md"])
