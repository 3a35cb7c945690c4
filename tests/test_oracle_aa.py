"""Pins of the oracle's average-atom pseudopotential (Sec. 2.4; oracle/aa.py):

  * the average atom is neutral in its Wigner-Seitz sphere;
  * at low temperature in a large sphere without xc it is the Thomas-Fermi
    atom, whose energy is -0.768745 Z^{7/3} Hartree;
  * the pseudo-density meets the paper's three constraints (value, slope and
    charge at r_cut), and the pseudopotential is continuous with -Z/r there;
  * the average atom solved in the pseudopotential reproduces the
    pseudo-density and the chemical potential (the pseudopotential is the
    potential whose response is the pseudo-density);
  * the radial Fourier transform against the closed form of a Gaussian.
"""
import math

import numpy as np
import pytest

from oracle import aa
from paper_2606_13283_amd import workloads as W


@pytest.fixture(scope="module")
def al10():
    rho = 1.0 / W.cell_length(1, 2.7) ** 3
    table, dE, d = aa.pseudopotential(13.0, rho, W.ev(10.0), 0.6, xc=True, dq=0.01, n_q=200)
    return table, dE, d


def test_neutral_and_constraints(al10):
    table, dE, d = al10
    A, P = d["aa"], d["pseudo"]
    g = A.grid
    r = g.r
    assert abs(g.integral(4 * math.pi * r * r * A.n) - 13.0) <= 1e-13 * 13.0
    i = int(np.searchsorted(r, P.r_cut))
    assert abs(P.n_pseudo[i] - A.n[i]) <= 1e-13 * A.n[i]
    # slope at r_cut: d/dr exp(a + b r^2 + c r^4) against the TF relation's n'
    slope = aa.density_slope(A)[i]
    s_ps = P.n_pseudo[i] * (2 * P.b * P.r_cut + 4 * P.c * P.r_cut ** 3)
    assert abs(s_ps - slope) <= 1e-11 * abs(slope)
    # the charge inside r_cut is conserved (same trapezoid rule on both)
    w = np.where(r <= P.r_cut, g.w, 0.0)
    w[i] *= 0.5
    q = lambda n: float(np.sum(w * 4 * math.pi * r * r * n))
    assert abs(q(P.n_pseudo) - q(A.n)) <= 1e-12 * q(A.n)
    # the pseudo-density is smooth at the nucleus where the true one is not
    assert P.n_pseudo[0] < 1e-6 * A.n[0]
    # continuity of the pseudopotential with -Z/r at r_cut
    assert abs(P.V_pseudo[i] + 13.0 / r[i]) <= 1e-10 * 13.0 / r[i]
    assert np.all(P.dV[r > P.r_cut] == 0.0)


def test_pseudo_atom_reproduces_pseudo_density(al10):
    table, dE, d = al10
    A, P = d["aa"], d["pseudo"]
    B = aa.solve(A.grid, 13.0, A.kT, P.V_pseudo, xc=True)
    assert np.max(np.abs(B.n - P.n_pseudo) / P.n_pseudo) <= 1e-9
    assert abs(B.mu - A.mu) <= 1e-9 * abs(A.mu)
    # the correction is the energy the smoothing removes: negative and large
    assert dE < -50.0


def test_thomas_fermi_atom_energy():
    Z = 10.0
    g = aa.RadialGrid.make(30.0, 4001, 1e-8)
    A = aa.solve(g, Z, 1e-3, -Z / g.r, xc=False)
    E = aa.energy(A, A.n, -Z / g.r)
    assert abs(E / (-0.768745 * Z ** (7.0 / 3.0)) - 1.0) <= 5e-3


def test_radial_transform_gaussian():
    # dV = exp(-r^2/(2 s^2)) inside a large radius: D(q) = (2 pi s^2)^{3/2} exp(-2 pi^2 s^2 q^2)
    s = 0.7
    g = aa.RadialGrid.make(12.0, 4001, 1e-8)
    A = aa.AverageAtom(g, 1.0, 0.1, False, -1.0 / g.r, np.ones_like(g.r), 0.0, np.zeros_like(g.r),
                       np.zeros_like(g.r), 0)
    P = aa.Pseudo(12.0, 0.0, 0.0, 0.0, np.ones_like(g.r), np.zeros_like(g.r), np.exp(-g.r ** 2 / (2 * s * s)))
    tab = aa.form_factor_table(A, P, 0.05, 30)
    q = np.arange(30) * 0.05
    ref = (2 * math.pi * s * s) ** 1.5 * np.exp(-2 * math.pi ** 2 * s * s * q * q)
    assert np.max(np.abs(tab - ref)) <= 1e-9 * ref[0]
