"""Pins of the oracle's tabulated local pseudopotential (eq. iepseudo with a
radial form factor given as samples of its non-Coulomb part D(q) = V(q) +
Z/(pi q^2)) and of an explicit Ewald splitting parameter (Sec. 2.6.3):

  * the local cubic reproduces any cubic polynomial exactly, and any even
    quadratic also on the first interval (where node -1 mirrors node 1), with
    its derivative;
  * the empty core given as a fine table equals the analytic empty core to the
    interpolation's accuracy (form factor, its derivative, the k = 0 limit);
  * with a non-analytic table, the forces are -dF/dR and the pressure
    -dF/dV by central finite differences (so the table enters the energy,
    the forces and the pressure consistently);
  * the Ewald energy does not depend on the splitting parameter.
"""
import math

import numpy as np
import pytest

from oracle import ionic, md, scf
from oracle.grid import Grid
from paper_2606_13283_amd import workloads as W

TOL = 1e-13


def smeared_core(Z, rc, sigma, dq, n):
    q = np.arange(n) * dq
    D = np.empty(n)
    D[0] = Z * math.pi * (2 * rc * rc + sigma * sigma)
    qq = q[1:]
    D[1:] = Z * (1.0 - np.cos(2 * math.pi * qq * rc) * np.exp(-(math.pi * qq * sigma) ** 2)) / (math.pi * qq * qq)
    return D


def test_cubic_interpolation_is_exact_for_cubics():
    dq = 0.05
    q_nodes = np.arange(40) * dq
    a, b, c, d = 0.7, -1.3, 0.4, 2.1
    tab = ionic.Tabulated(a + b * q_nodes + c * q_nodes ** 2 + d * q_nodes ** 3, dq)
    q = np.random.default_rng(0).uniform(dq, 36 * dq, 500)
    v, dv = tab.interpolate(q)
    assert np.max(np.abs(v - (a + b * q + c * q ** 2 + d * q ** 3))) <= 1e-12
    assert np.max(np.abs(dv - (b + 2 * c * q + 3 * d * q ** 2))) <= 1e-10
    # even quadratic: exact on the first interval too (mirrored node -1)
    tab2 = ionic.Tabulated(a + c * q_nodes ** 2, dq)
    q0 = np.linspace(0.0, dq, 17)[:-1]
    v0, dv0 = tab2.interpolate(q0)
    assert np.max(np.abs(v0 - (a + c * q0 ** 2))) <= 1e-13
    assert np.max(np.abs(dv0 - 2 * c * q0)) <= 1e-11
    # at the nodes the table's own values come back
    vn, _ = tab.interpolate(q_nodes[:37])
    assert np.max(np.abs(vn - tab.table[:37])) <= 1e-13


def test_table_too_short_is_an_error():
    tab = ionic.Tabulated(np.zeros(10), 0.1)
    with pytest.raises(ValueError):
        tab.interpolate(np.array([0.85]))  # the cubic around x = 8.5 needs node 10


def test_fine_empty_core_table_equals_analytic():
    g = Grid((15.3, 15.3, 18.0), (32, 32, 36))
    Z, rc, dq = 3.0, 1.1, 0.002
    n = int(g.kabs.max() / dq) + 8
    tab = ionic.Tabulated(smeared_core(Z, rc, 0.0, dq, n), dq)
    Va = ionic.form_factor(g, Z, rc)
    Vt = ionic.form_factor(g, Z, tab)
    nz = g.nonzero
    assert np.max(np.abs(Vt[nz] - Va[nz]) / np.abs(Z / (math.pi * g.k2[nz]))) <= 2e-9
    Da = ionic.form_factor_dq(g, Z, rc)
    Dt = ionic.form_factor_dq(g, Z, tab)
    assert np.max(np.abs(Dt[nz] - Da[nz]) / np.abs(2 * Z / (math.pi * g.kabs[nz] ** 3))) <= 5e-6
    assert abs(ionic.form_factor_k0(Z, tab) - ionic.form_factor_k0(Z, rc)) <= 1e-14 * 2 * math.pi * Z * rc * rc


@pytest.fixture(scope="module")
def tab_base():
    L = W.cell_length(4, 2.7)
    pos = W.random_positions(4, L, 1.8897, np.random.default_rng(11))
    dq = 0.004
    n = int(math.sqrt(3) * 8 / L / dq) + 16
    tab = ionic.Tabulated(smeared_core(3.0, 1.1, 0.45, dq, n), dq)
    s = scf.System((L, L, L), (16, 16, 16), pos, np.zeros(4, int), (3.0,), (tab,), (W.AL_MASS,), W.ev(10.0),
                   0.2, True)
    return s, md.solve_at(s, tol=TOL, solver="anderson")


def _F_at(s, prev_n, pos=None, cell=None):
    if cell is not None:
        s = scf.System(cell, s.shape, pos, s.species, s.Z, s.rc, s.mass, s.kT, s.lam, s.xc)
    elif pos is not None:
        s = s.with_positions(pos)
    # the solution alone is needed: Anderson's acceleration reaches the same
    # fixed point (test_one_fixed_point_for_all_algorithms) in fewer iterations
    r = md.solve_at(s, init="given", prev=prev_n, tol=TOL, solver="anderson")
    assert r.scf.converged
    return r.th.F


def test_tabulated_forces_are_minus_gradient(tab_base):
    s, r = tab_base
    assert r.scf.converged
    h = 1e-4
    for j, a in ((0, 1), (2, 0)):
        p = s.pos.copy(); p[j, a] += h
        m = s.pos.copy(); m[j, a] -= h
        fnum = -(_F_at(s, r.scf.n, p) - _F_at(s, r.scf.n, m)) / (2 * h)
        assert abs(fnum - r.th.forces[j, a]) <= 2e-7 * max(1.0, np.max(np.abs(r.th.forces)))


def test_tabulated_pressure_is_minus_volume_derivative(tab_base):
    s, r = tab_base
    h = 2e-5
    frac = s.pos / np.array(s.cell)
    Fs = []
    for f in (1 + h, 1 - h):
        cell = tuple(c * f for c in s.cell)
        Fs.append(_F_at(s, r.scf.n / f ** 3, frac * np.array(cell), cell))
    V = s.grid.volume
    P_num = -(Fs[0] - Fs[1]) / (V * ((1 + h) ** 3 - (1 - h) ** 3))
    assert abs(P_num - r.th.P) <= 1e-7 * abs(r.th.P) + 1e-10


def test_ewald_energy_independent_of_alpha():
    L = W.cell_length(8, 2.7)
    pos = W.random_positions(8, L, 1.8897, np.random.default_rng(5))
    g = Grid((L, L, L), (48, 48, 48))
    Zj = np.full(8, 3.0)
    S = ionic.structure_factors(g, pos, np.zeros(8, int), 1)
    SZ = ionic.charge_structure_factor(S, (3.0,))
    a0 = ionic.ewald_alpha(g)
    U = [ionic.ewald(g, pos, Zj, SZ, alpha=a0 * f)["U_ii"] for f in (0.9, 1.0, 1.15)]
    assert max(U) - min(U) <= 1e-9 * abs(U[1])
