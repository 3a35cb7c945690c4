"""Pins for the oracle's SCF, energies, pressure and forces: the More weight
closed form, charge conservation, one fixed point for every algorithm,
forces and pressure as finite differences of the free energy, translation
and lattice symmetry, and the exactness of the one-center guess for one atom.
"""
import math

import numpy as np
import pytest

from oracle import fd, ionic, md, scf, thermo
from oracle.grid import Grid
from paper_2606_13283_amd import workloads as W

TOL = 1e-13


def small_system(T_ev=10.0, seed=11, n_atoms=4, N=16, lam=0.2, xc=True):
    L = W.cell_length(n_atoms, 2.7)
    pos = W.random_positions(n_atoms, L, 1.8897, np.random.default_rng(seed))
    return scf.System((L, L, L), (N, N, N), pos, np.zeros(n_atoms, int), (3.0,), (1.1,),
                      (W.AL_MASS,), W.ev(T_ev), lam, xc)


@pytest.fixture(scope="module")
def base():
    # the fixed point itself; the paper's iteration from the uniform density
    # reaches it too (test_one_fixed_point_for_all_algorithms)
    s = small_system()
    return s, md.solve_at(s, tol=TOL, solver="anderson")


def test_charge_conservation(base):
    s, r = base
    assert r.scf.converged
    assert abs(s.grid.integrate(r.scf.n) - s.Ne) <= 1e-13 * s.Ne


def test_more_weight_closed_form():
    # jellium (V^ie = 0), TF + Hartree only, one cosine perturbation of wavevector G:
    # w = chi (4 pi/G^2) / (1 + chi 4 pi/G^2), and one step lands on the uniform fixed point
    L, N = 10.0, 16
    n0 = 0.03
    Ne = n0 * L ** 3
    s = scf.System((L, L, L), (N, N, N), np.zeros((1, 3)), np.zeros(1, int), (Ne,), (0.0,), (1.0,),
                   W.ev(5.0), 0.0, False)
    ion = scf.Ionic(np.zeros((1, N, N, N), complex), np.zeros((N, N, N), complex), np.zeros((N, N, N)))
    x = s.grid.points()[..., 0]
    eps = 1e-6
    n_i = n0 * (1 + eps * np.cos(2 * math.pi * 2 * x / L))
    eta0 = fd.I_p12_inverse(n0 / fd.c_n(s.kT))
    chi = fd.c_n(s.kT) / (2 * s.kT) * fd.I_m12(np.array([eta0]))[0]
    G = 2 * math.pi * 2 / L
    g_ = chi * 4 * math.pi / G ** 2
    # the secant weight (default) and the weight exactly as printed agree here
    for mixing in ("more", "more_printed"):
        r = scf.scf(s, ion, n_i, mixing=mixing, warmup=0, more_trust=1e30, max_iter=1, tol=0.0)
        assert abs(r.weights[0] - g_ / (1 + g_)) <= 1e-5, mixing
        n_o = r.n + r.weights[0] * (n_i - r.n)
        assert np.max(np.abs(n_o - n0)) <= 1e-3 * eps * n0, mixing


def test_one_fixed_point_for_all_algorithms(base):
    s, r = base  # r: Anderson's acceleration from the uniform density
    ion = r.ion
    # the paper's iteration (Sec. 2.5, More's weight) from the uniform density
    rp = scf.scf(s, ion, scf.initial_density(s, ion)[0], mixing="more", tol=TOL)
    assert r.scf.iters < rp.iters
    pert = r.scf.n * (1 + 0.05 * np.cos(2 * math.pi * s.grid.points()[..., 1] / s.cell[1]))
    pert *= s.Ne / s.grid.integrate(pert)
    # fixed mixing and More's weight from a perturbed density (a residual of
    # 1e-11 leaves F within 1e-20, P and forces within 1e-11)
    rf = scf.scf(s, ion, pert, mixing="fixed", w_fixed=0.9, tol=1e-11)
    rg = scf.scf(s, ion, pert, mixing="more", tol=1e-11)
    for other in (rp, rf, rg):
        assert other.converged
        th = thermo.evaluate(s, ion, other)
        assert abs(th.F - r.th.F) <= 1e-12 * abs(r.th.F)
        assert abs(th.P - r.th.P) <= 1e-10 * abs(r.th.P)
        assert np.max(np.abs(th.forces - r.th.forces)) <= 1e-9 * max(np.max(np.abs(r.th.forces)), 1e-6)


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


def test_forces_are_minus_gradient(base):
    s, r = base
    h = 1e-4
    for j, a in ((1, 0), (3, 2)):
        p = s.pos.copy(); p[j, a] += h
        m = s.pos.copy(); m[j, a] -= h
        fnum = -(_F_at(s, r.scf.n, p) - _F_at(s, r.scf.n, m)) / (2 * h)
        assert abs(fnum - r.th.forces[j, a]) <= 2e-7 * max(1.0, np.max(np.abs(r.th.forces)))
    # (the total force is not zero: the grid breaks translation invariance, the egg-box effect)


def test_pressure_is_minus_volume_derivative(base):
    s, r = base
    h = 2e-5
    frac = s.pos / np.array(s.cell)
    Fs = []
    for f in (1 + h, 1 - h):
        cell = tuple(c * f for c in s.cell)
        Fs.append(_F_at(s, r.scf.n / f ** 3, frac * np.array(cell), cell))
    V = s.grid.volume
    P_num = -(Fs[0] - Fs[1]) / (V * ((1 + h) ** 3 - (1 - h) ** 3))
    assert abs(P_num - r.th.P) <= 1e-7 * abs(r.th.P) + 1e-10


def test_translation_by_grid_vector(base):
    s, r = base
    shift = np.array([3, 5, 14]) * np.array(s.cell) / np.array(s.shape)
    r2 = md.solve_at(s.with_positions(s.pos + shift), tol=TOL, solver="anderson")
    assert abs(r2.th.F - r.th.F) <= 1e-12 * abs(r.th.F)
    assert abs(r2.th.P - r.th.P) <= 1e-11 * abs(r.th.P)
    assert np.max(np.abs(r2.th.forces - r.th.forces)) <= 1e-9
    rolled = np.roll(r.scf.n, (3, 5, 14), axis=(0, 1, 2))
    assert np.max(np.abs(r2.scf.n - rolled)) <= 1e-10 * np.max(r.scf.n)


def test_perfect_fcc_on_grid_has_zero_forces():
    L = W.cell_length(32, 2.7)
    pos = W.fcc_positions(2, L)
    s = scf.System((L, L, L), (16, 16, 16), pos, np.zeros(32, int), (3.0,), (1.1,), (W.AL_MASS,),
                   W.ev(10.0), 0.2, True)
    r = md.solve_at(s, tol=TOL, solver="anderson")
    assert r.scf.converged
    # inversion symmetry about every atom: the electron-ion and reciprocal Ewald forces vanish
    assert np.max(np.abs(r.th.force_terms["F_ie"])) <= 1e-10
    assert np.max(np.abs(r.th.force_terms["F_pm"])) <= 1e-10
    # the real-space Ewald sum keeps one of two equidistant images at separation L/2, so F_pp
    # is bounded by the minimum-image truncation, erfc(alpha L/2) scale
    a = r.th.terms["alpha"]
    from scipy.special import erfc
    d = L / 2
    bound = 4 * 9.0 * (erfc(a * d) / d + 2 * a / math.sqrt(math.pi) * math.exp(-(a * d) ** 2)) / d
    assert np.max(np.abs(r.th.force_terms["F_pp"])) <= bound
    assert abs(r.th.P_terms["P_ii"] - r.th.terms["U_ii"] / (3 * L ** 3)) <= 1e-15


def test_one_center_exact_for_single_atom():
    g = Grid((9.0, 9.0, 9.0), (24, 24, 24))
    s = scf.System(g.cell, g.shape, np.array([[1.0, 2.0, 3.0]]), np.zeros(1, int), (3.0,), (1.1,),
                   (1.0,), W.ev(10.0), 0.2, True)
    sigma = 2.5  # wide enough that the guess floor (1e-3 n0) never binds
    def gauss_hat(r0):
        kr = g.k[0] * r0[0] + g.k[1] * r0[1] + g.k[2] * r0[2]
        return 3.0 * np.exp(-2 * math.pi ** 2 * sigma ** 2 * g.k2) * np.exp(-2j * math.pi * kr)
    r0 = np.array([1.0, 2.0, 3.0])
    r1 = np.array([4.3, 0.2, 6.6])
    S0 = ionic.structure_factors(g, r0[None], np.zeros(1, int), 1)
    ion1 = scf.ionic_setup(s.with_positions(r1[None]))
    n1, fb = scf.initial_density(s.with_positions(r1[None]), ion1, "one_center", (gauss_hat(r0), 3.0 * S0[0]))
    assert not fb
    ref = g.inverse(gauss_hat(r1))
    assert np.min(ref) > 2 * scf.GUESS_FLOOR * s.Ne / g.volume
    assert np.max(np.abs(n1 - ref)) <= 1e-12 * np.max(ref)
