"""Writes the stored expected values of the full-size parity tests.

Every value here comes from the FP64 CPU oracle (`oracle/`) solving the seeded
workload itself; nothing is read from the HIP path.  The inputs come from the
seeded input generators (`paper_2606_13283_amd/workloads.py`, which holds none
of the method's arithmetic).

    python tests/golden/make_goldens.py fcc32 fcc256 rand1024 rand4000 fcc256_md

Each name writes tests/golden/oracle_<name>.json:
  static workloads: the SCF fixed point (Sec. 2.5; reached from the uniform
    density by the oracle's Anderson-accelerated iteration) to a relative
    residual of 1e-12, then F, E, P and every term (Sec. 2.6), mu, forces
    (eq. force; all atoms, or a seeded sample of atoms on the largest cell),
    and the converged density at a seeded sample of grid points (every point
    of the 32-atom cell, whose 1 eV electrons the oracle solves with the
    paper's own iteration);
  fcc256_md: the 256-atom fcc cell's Verlet trajectory (Sec. 2.1) for three
    steps after the initial solve, each step's SCF started from the one-center
    guess (Sec. 2.5.1) of the previous step: positions, velocities, F, P, mu and
    all forces per step, and whether the guess fell back to the uniform
    density.
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


def static(name, paper_iteration=False, full_density=False):
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
    if paper_iteration:
        # the paper's own iteration (More mixing), where Anderson's acceleration
        # converges slowly (degenerate electrons at 1 eV)
        res = oscf.scf(s, ion, n0, mixing="more", tol=TOL, w_fixed=w.w_fixed, max_iter=5000)
    else:
        # the fixed point by Anderson's acceleration: the same answer as the paper's
        # iteration (pinned on small cells) in a fraction of the oracle's time
        res = oscf.scf_anderson(s, ion, n0, tol=TOL, beta=0.3, max_iter=1000)
    t_scf = time.time() - t0
    assert res.converged, name
    from oracle import thermo
    th = thermo.evaluate(s, ion, res, forces=True, atoms=atoms)
    idx = np.arange(int(np.prod(s.shape))) if full_density else sample_points(s.shape, 11)
    out = dict(workload=w.name, grid=list(w.grid), cell=list(w.cell), scf_tol=TOL, init="uniform",
               w_fixed=w.w_fixed, residual=res.residual, mu=res.mu,
               **thermo_dict(th),
               force_atoms=list(range(n_atoms)) if atoms is None else atoms,
               forces=th.forces.tolist(),
               density_index=idx.tolist(), density=res.n.reshape(-1)[idx].tolist(),
               oracle_seconds=dict(ionic_setup=t_ion, scf=t_scf))
    if paper_iteration:
        out.update(oracle_iteration="more", oracle_iters=res.iters)
    else:
        out.update(oracle_iters_anderson=res.iters)
    return out


def solve_step(s, init, prev):
    """One MD step's solve: initial density (uniform, or the one-center guess
    of Sec. 2.5.1 from the previous step's converged spectrum and S_Z), the
    fixed point by the Anderson-accelerated iteration, F, P and forces."""
    from oracle import thermo
    ion = oscf.ionic_setup(s)
    n0, fb = oscf.initial_density(s, ion, init, prev)
    res = oscf.scf_anderson(s, ion, n0, tol=TOL, beta=0.3, max_iter=1000)
    assert res.converged
    th = thermo.evaluate(s, ion, res)
    return ion, res, th, fb


def fcc256_md(steps=3):
    w = W.fcc256()
    s = system_of(w)
    m = omd.masses(s)
    dt = w.dt
    ion, res, th, _ = solve_step(s, "uniform", None)
    out = dict(workload=w.name, grid=list(w.grid), cell=list(w.cell), scf_tol=TOL, dt=dt,
               init="one_center", w_fixed=w.w_fixed, start=dict(pos=s.pos.tolist(), vel=w.vel.tolist(),
                                                                F=th.F, P=th.P, mu=res.mu,
                                                                forces=th.forces.tolist()),
               steps=[])
    r_prev = omd.verlet_start(s.pos, w.vel, th.forces, m, dt)
    r_cur, F_cur = s.pos, th.forces
    prev = (s.grid.forward(res.n), ion.SZ)
    for step in range(steps):
        r_next, v = omd.verlet_step(r_cur, r_prev, F_cur, m, dt)
        s_next = s.with_positions(r_next)
        ion, res, th, fb = solve_step(s_next, "one_center", prev)
        out["steps"].append(dict(pos=r_next.tolist(), vel=v.tolist(), F=th.F, E=th.E, P=th.P, mu=res.mu,
                                 forces=th.forces.tolist(), guess_fallback=bool(fb)))
        print("fcc256_md step %d: fallback %s, F %.15g" % (step, fb, th.F), flush=True)
        r_prev, r_cur, F_cur = r_cur, r_next, th.forces
        prev = (s.grid.forward(res.n), ion.SZ)
    return out


def main(names):
    for name in names:
        t0 = time.time()
        if name == "fcc256_md":
            out = fcc256_md()
        elif name == "fcc32":
            out = static(name, paper_iteration=True, full_density=True)
        else:
            out = static(name)
        path = os.path.join(HERE, "oracle_%s.json" % name)
        with open(path, "w") as f:
            json.dump(out, f, indent=0)
        print("%s: written in %.0f s" % (path, time.time() - t0), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["fcc32", "fcc256", "rand1024", "rand4000", "fcc256_md"])
