"""Pins of the oracle's stress tensor (Sec. 2.6; oracle/stress.py):

  * each term's trace against the pressure term computed from its own,
    independent formula (P_vW = 2 F_vW/(3|Omega|), P_H = E_H/(3|Omega|), the
    electron-ion pressure of Sec. 2.6.5, the ideal-gas and xc pressures; the
    Ewald trace against U^ii/(3|Omega|) to truncation; the ions' kinetic
    trace against 2 K^i/(3|Omega|));
  * the diagonal of the total tensor against central finite differences of the
    free energy under a strain of one cell edge at fixed fractional positions
    (alpha held fixed, SCF re-converged), on an orthorhombic cell whose three
    diagonal entries differ; the ion-ion tensor alone against finite
    differences of U^ii;
  * the off-diagonal entries through rotation: a cubic cell turned by 90
    degrees about z (a grid symmetry) must give R sigma R^T term by term;
    every term is symmetric.
"""
import math

import numpy as np
import pytest

from oracle import ionic, scf, stress, thermo
from paper_2606_13283_amd import workloads as W

TOL = 1e-13


def solve(s, n_init=None):
    ion = scf.ionic_setup(s)
    n0 = n_init if n_init is not None else scf.initial_density(s, ion)[0]
    r = scf.scf_anderson(s, ion, n0, tol=TOL, beta=0.3)
    assert r.converged
    return ion, r


def ortho_system(alpha=None):
    L = W.cell_length(6, 2.7)
    cell = (0.9 * L, 1.0 * L, 1.15 * L)
    pos = W.random_positions(6, cell, 1.8897, np.random.default_rng(17))
    s = scf.System(cell, (16, 18, 20), pos, np.zeros(6, int), (3.0,), (1.1,), (W.AL_MASS,), W.ev(8.0), 0.2, True)
    if alpha is not None:
        s.ewald_alpha = alpha
    return s


@pytest.fixture(scope="module")
def base():
    s = ortho_system()
    s.ewald_alpha = ionic.ewald_alpha(s.grid)  # held fixed under strain
    ion, r = solve(s)
    th = thermo.evaluate(s, ion, r)
    vel = np.random.default_rng(3).normal(0, math.sqrt(s.kT / W.AL_MASS), s.pos.shape)
    terms = stress.stress(s, ion, r, vel=vel)
    return s, ion, r, th, vel, terms


def test_traces_match_pressure_terms(base):
    s, ion, r, th, vel, T = base
    V = s.grid.volume
    tr = {k: -np.trace(v) / 3.0 for k, v in T.items()}
    P = th.P_terms
    assert abs(tr["TF"] - P["P_TF"]) <= 1e-13 * abs(P["P_TF"])
    assert abs(tr["vW"] - P["P_vW"]) <= 1e-12 * abs(P["P_vW"])
    assert abs(tr["xc"] - P["P_xc"]) <= 1e-13 * abs(P["P_xc"])
    assert abs(tr["ee"] - P["P_H"]) <= 1e-12 * abs(P["P_H"])
    assert abs(tr["ie"] - P["P_ie"]) <= 1e-12 * abs(P["P_ie"])
    # U^ii/(3|Omega|) takes U^ii as independent of alpha; the printed tensor holds
    # alpha fixed: they agree to the Ewald truncation, ~exp(-pi N/4) at N = 16
    assert abs(tr["ii"] - P["P_ii"]) <= 2e-5 * abs(P["P_ii"])
    assert abs(tr["i"] - 2.0 * thermo.ion_kinetic(s, vel) / (3.0 * V)) <= 1e-14 * abs(tr["i"])
    for k, v in T.items():
        assert np.max(np.abs(v - v.T)) <= 1e-14 * max(np.max(np.abs(v)), 1e-30), k


def _strained(s, axis, f):
    cell = list(s.cell)
    cell[axis] *= f
    frac = s.pos / np.array(s.cell)
    return scf.System(tuple(cell), s.shape, frac * np.array(cell), s.species, s.Z, s.rc, s.mass, s.kT, s.lam,
                      s.xc, s.ewald_alpha)


def test_diagonal_is_strain_derivative_of_F(base):
    s, ion, r, th, vel, T = base
    tot = sum(T[k] for k in stress.TERMS if k != "i")
    assert len({round(tot[a, a], 9) for a in range(3)}) == 3  # the diagonal entries differ
    h = 2e-5
    for axis in range(3):
        Fs = []
        for f in (1 + h, 1 - h):
            s2 = _strained(s, axis, f)
            ion2, r2 = solve(s2, r.n / f)
            Fs.append(thermo.evaluate(s2, ion2, r2, forces=False).F)
        dF = (Fs[0] - Fs[1]) / (2 * h)
        sig = dF / s.grid.volume
        assert abs(sig - tot[axis, axis]) <= 1e-7 * np.max(np.abs(tot)), (axis, sig, tot[axis, axis])


def test_ion_ion_tensor_is_strain_derivative_of_Uii(base):
    s, ion, r, th, vel, T = base
    h = 1e-5
    for axis in range(3):
        U = []
        for f in (1 + h, 1 - h):
            s2 = _strained(s, axis, f)
            g = s2.grid
            S = ionic.structure_factors(g, s2.pos, s2.species, 1)
            U.append(ionic.ewald(g, s2.pos, s2.Zj, ionic.charge_structure_factor(S, s2.Z),
                                 alpha=s.ewald_alpha, atoms=[])["U_ii"])
        sig = (U[0] - U[1]) / (2 * h) / s.grid.volume
        assert abs(sig - T["ii"][axis, axis]) <= 1e-8 * np.max(np.abs(T["ii"])), axis


def _rotated(s, pos, vel, M):
    L = s.cell[0]
    s2 = s.with_positions((pos @ M.T) % L)
    return s2, vel @ M.T


def test_axis_swap_and_rotation_transform_every_term():
    """Swapping x and y maps the grid and the reciprocal box onto themselves, so
    sigma' = P sigma P^T holds to rounding.  A 90-degree turn about z maps the
    grid onto itself but not the box's Nyquist planes (+N/2 only), so it holds
    to the Nyquist-plane error of the discretisation; the off-diagonal entries
    flip sign under it, which the swap cannot show."""
    L = W.cell_length(5, 2.7)
    pos = W.random_positions(5, L, 1.8897, np.random.default_rng(23))
    s = scf.System((L, L, L), (16, 16, 16), pos, np.zeros(5, int), (3.0,), (1.1,), (W.AL_MASS,), W.ev(10.0),
                   0.2, True)
    vel = np.random.default_rng(4).normal(0, 1e-3, pos.shape)
    ion, r = solve(s)
    A = stress.stress(s, ion, r, vel=vel)
    tot = stress.total(A)
    off = np.max(np.abs(tot - np.diag(np.diag(tot))))
    assert off > 1e-2 * np.max(np.abs(tot))  # the off-diagonal entries are not small
    P = np.array([[0.0, 1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    for M, tol in ((P, 1e-10), (R, 1e-3)):
        s2, vel2 = _rotated(s, pos, vel, M)
        ion2, r2 = solve(s2)
        B = stress.stress(s2, ion2, r2, vel=vel2)
        for k in stress.TERMS:
            want = M @ A[k] @ M.T
            scale = max(np.max(np.abs(A[k])), 1e-12)
            assert np.max(np.abs(B[k] - want)) <= tol * scale, (k, tol, B[k], want)
