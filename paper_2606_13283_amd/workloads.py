"""Seeded synthetic inputs (aluminium state points) shared by the tests, the
benchmark and the oracle's callers.

This module holds no arithmetic of the method: it only builds cells,
positions, velocities, temperatures and grid sizes from seeds, with the
constants needed to express them in Hartree atomic units.  It imports nothing
from the rest of the package.

Workloads (all Al, Z = 3, empty-core radius 1.1 bohr, TF + 0.2 vW + LDA):
  fcc32     32 atoms, fcc 2x2x2 at 2.7 g/cm^3, each coordinate perturbed by a
            seeded Gaussian of 0.05 Angstrom, 32^3 grid, T = 1 eV, seed 1
  fcc256    256 atoms, fcc 4x4x4 at 2.7 g/cm^3 (atoms on grid points), 64^3,
            T = 5 eV, Maxwell-Boltzmann velocities, seed 2, 0.2 fs steps
  batch64   64 snapshots of 108 atoms, density U[1.5, 5.4] g/cm^3, T log-uniform
            in [1, 20] eV, grid 48..72 per side at spacing ~0.38 bohr, random
            positions with 1.0 Angstrom minimum separation, seed 3000 + i
  rand1024  1024 atoms at 2.7 g/cm^3, 128^3, T = 10 eV, random positions with
            1.0 Angstrom minimum separation, MB velocities, seed 5
  rand4000  4000 atoms at 2.7 g/cm^3, 192^3, T = 10 eV, seed 6
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# CODATA 2018
HARTREE_EV = 27.211386245988
BOHR_ANGSTROM = 0.529177210903
BOHR_CM = BOHR_ANGSTROM * 1e-8
AU_TIME_S = 2.4188843265857e-17
ELECTRON_MASSES_PER_DALTON = 1822.888486209
DALTON_G = 1.66053906660e-24
AL_MASS_DALTON = 26.9815385

AL_Z = 3.0
AL_RC = 1.1  # bohr
AL_MASS = AL_MASS_DALTON * ELECTRON_MASSES_PER_DALTON  # electron masses
DT_02FS = 0.2e-15 / AU_TIME_S  # 0.2 fs in atomic time units


def ev(x: float) -> float:
    return x / HARTREE_EV


def cell_length(n_atoms: int, rho_g_cm3: float) -> float:
    """Cubic cell edge (bohr) holding n_atoms Al at mass density rho."""
    n_ion_cm3 = rho_g_cm3 / (AL_MASS_DALTON * DALTON_G)
    n_ion_bohr3 = n_ion_cm3 * BOHR_CM ** 3
    return (n_atoms / n_ion_bohr3) ** (1.0 / 3.0)


def fcc_positions(cells: int, L: float) -> np.ndarray:
    a = L / cells
    basis = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    pts = []
    for i in range(cells):
        for j in range(cells):
            for k in range(cells):
                for b in basis:
                    pts.append((np.array([i, j, k]) + b) * a)
    return np.array(pts, dtype=np.float64)


def random_positions(n: int, L, dmin: float, rng: np.random.Generator) -> np.ndarray:
    """Uniform positions in the cell [0, L) (L a scalar or three edges), rejecting
    any closer than dmin to an earlier one (minimum image)."""
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    pos = np.empty((n, 3))
    k = 0
    tries = 0
    while k < n:
        p = rng.uniform(0.0, 1.0, 3) * L
        if k:
            d = pos[:k] - p
            d -= L * np.round(d / L)
            if np.min(np.einsum("ij,ij->i", d, d)) < dmin * dmin:
                tries += 1
                if tries > 1000 * n:
                    raise RuntimeError("cannot place atoms at this separation")
                continue
        pos[k] = p
        k += 1
    return pos


def mb_velocities(n: int, kT: float, mass: float, rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(0.0, math.sqrt(kT / mass), size=(n, 3))
    v -= v.mean(axis=0)
    return v


def smooth_even(n: int) -> int:
    """Smallest even integer >= n whose only prime factors are 2, 3, 5."""
    m = max(2, int(math.ceil(n)))
    while True:
        if m % 2 == 0:
            r = m
            for p in (2, 3, 5):
                while r % p == 0:
                    r //= p
            if r == 1:
                return m
        m += 1


@dataclass
class Workload:
    name: str
    cell: tuple
    grid: tuple
    pos: np.ndarray
    kT: float
    vel: np.ndarray | None = None
    dt: float = DT_02FS
    steps: int = 1
    species: np.ndarray = field(default=None)
    Z: tuple = (AL_Z,)
    rc: tuple = (AL_RC,)
    mass: tuple = (AL_MASS,)
    lam: float = 0.2
    xc: bool = True
    seed: int = 0
    w_fixed: float = 0.95  # fixed mixing weight before More's weight switches on

    def __post_init__(self):
        if self.species is None:
            self.species = np.zeros(self.pos.shape[0], dtype=np.int32)


def fcc32(seed: int = 1) -> Workload:
    L = cell_length(32, 2.7)
    rng = np.random.default_rng(seed)
    pos = fcc_positions(2, L) + rng.normal(0.0, 0.05 / BOHR_ANGSTROM, size=(32, 3))
    return Workload("fcc32_32^3_1eV", (L, L, L), (32, 32, 32), pos, ev(1.0),
                    vel=np.zeros((32, 3)), steps=1, seed=seed, w_fixed=0.99)


def fcc256(seed: int = 2, steps: int = 50) -> Workload:
    L = cell_length(256, 2.7)
    rng = np.random.default_rng(seed)
    pos = fcc_positions(4, L)
    kT = ev(5.0)
    vel = mb_velocities(256, kT, AL_MASS, rng)
    return Workload("fcc256_64^3_5eV", (L, L, L), (64, 64, 64), pos, kT, vel=vel, steps=steps,
                    seed=seed)


def fcc256_at(T_ev: float, seed: int, steps: int = 50) -> Workload:
    """The 256-atom fcc cell at 2.7 g/cm^3 and 64^3 at temperature T_ev (eV), with
    Maxwell-Boltzmann velocities from `seed`: the trajectories the learned
    initial density is trained and evaluated on."""
    L = cell_length(256, 2.7)
    rng = np.random.default_rng(seed)
    pos = fcc_positions(4, L)
    kT = ev(T_ev)
    vel = mb_velocities(256, kT, AL_MASS, rng)
    return Workload("fcc256_64^3_%geV" % T_ev, (L, L, L), (64, 64, 64), pos, kT, vel=vel, steps=steps, seed=seed,
                    w_fixed=0.99 if T_ev < 3.0 else 0.95)


def batch_snapshot(i: int) -> Workload:
    seed = 3000 + i
    rng = np.random.default_rng(seed)
    rho = rng.uniform(1.5, 5.4)
    T = math.exp(rng.uniform(math.log(1.0), math.log(20.0)))
    L = cell_length(108, rho)
    N = min(max(smooth_even(L / 0.38), 48), 72)
    pos = random_positions(108, L, 1.0 / BOHR_ANGSTROM, rng)
    return Workload("batch108_%d" % i, (L, L, L), (N, N, N), pos, ev(T), seed=seed)


def batch64(count: int = 64):
    return [batch_snapshot(i) for i in range(count)]


def rand1024(seed: int = 5, steps: int = 100) -> Workload:
    L = cell_length(1024, 2.7)
    rng = np.random.default_rng(seed)
    pos = random_positions(1024, L, 1.0 / BOHR_ANGSTROM, rng)
    kT = ev(10.0)
    vel = mb_velocities(1024, kT, AL_MASS, rng)
    return Workload("rand1024_128^3_10eV", (L, L, L), (128, 128, 128), pos, kT, vel=vel,
                    steps=steps, seed=seed, w_fixed=0.97)


def rand4000(seed: int = 6) -> Workload:
    L = cell_length(4000, 2.7)
    rng = np.random.default_rng(seed)
    pos = random_positions(4000, L, 1.0 / BOHR_ANGSTROM, rng)
    return Workload("rand4000_192^3_10eV", (L, L, L), (192, 192, 192), pos, ev(10.0), seed=seed,
                    w_fixed=0.98)


def small_random(n_atoms: int, N: int, rho: float, T_ev: float, seed: int,
                 shape=None, stretch=(1.0, 1.0, 1.0)) -> Workload:
    """Small seeded random-position cell for parity tests (optionally orthorhombic)."""
    L = cell_length(n_atoms, rho)
    cell = tuple(L * s for s in stretch)
    rng = np.random.default_rng(seed)
    pos = random_positions(n_atoms, cell, 1.0 / BOHR_ANGSTROM, rng)
    grid = shape if shape is not None else (N, N, N)
    return Workload("rand%d_%s_%geV" % (n_atoms, "x".join(map(str, grid)), T_ev), cell, grid, pos,
                    ev(T_ev), vel=np.zeros((n_atoms, 3)), seed=seed)
