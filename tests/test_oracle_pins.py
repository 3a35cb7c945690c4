"""Closed-form pins of the oracle's von Weizsaecker term and of the one-center
guess's floor and fallback branches.

von Weizsaecker (the gradient correction of Sec. 2.2; standard form
F_vW = (lambda/2) int |grad sqrt n|^2, v_vW = -(lambda/2) lap(sqrt n)/sqrt n):
  * sqrt n = a + b x (periodic Gaussian of width sigma): int |grad s|^2 =
    b^2 (3/2) pi^{3/2} sigma for one image in the cell (real-space integral,
    no Fourier sum involved), and lap s from the analytic second derivative of
    the images;
  * n = n0 (1 + eps cos(G x)): F_vW = (lambda/8) n0 G^2 |Omega| (1 - sqrt(1 - eps^2))
    exactly (the angular average of sin^2 / (1 + eps cos)), and the pointwise
    potential from the chain rule.
A common factor error on F_vW or v_vW (which finite differences of F cannot
see, since forces and pressure scale with it) fails these.

One-center guess (Sec. 2.5.1, with the floor / fallback reading): a radial
profile with a negative ring, superposed on one atom, against the brute-force
real-space image sum of the same profile at the new position.
"""
import math

import numpy as np

from oracle import functional as fn
from oracle import ionic, scf
from oracle.grid import Grid
from paper_2606_13283_amd import workloads as W


def _images(g, r0, f):
    """sum over the 27 nearest periodic images of f(d2, d), d = r - r0 - R."""
    P = g.points()
    acc = np.zeros(g.shape)
    for ix in (-1, 0, 1):
        for iy in (-1, 0, 1):
            for iz in (-1, 0, 1):
                R = np.array([ix * g.cell[0], iy * g.cell[1], iz * g.cell[2]])
                d = P - r0 - R
                acc += f(np.sum(d * d, axis=-1))
    return acc


def test_vw_gaussian_sqrt_density_closed_form():
    L, N = 12.0, 48  # h = 0.25, sigma = 4 h; images overlap at the e^{-36} level
    g = Grid((L, L, L), (N, N, N))
    sigma, a, b, lam = 1.0, 0.3, 0.7, 0.2
    r0 = np.array([5.1, 6.3, 4.4])
    gauss = _images(g, r0, lambda d2: np.exp(-d2 / (2 * sigma ** 2)))
    lap = _images(g, r0, lambda d2: (d2 / sigma ** 4 - 3 / sigma ** 2) * np.exp(-d2 / (2 * sigma ** 2)))
    s = a + b * gauss
    v, F = fn.vw_terms(g, s * s, lam)
    F_ref = 0.5 * lam * b * b * 1.5 * math.pi ** 1.5 * sigma
    assert abs(F - F_ref) <= 1e-12 * F_ref
    v_ref = -0.5 * lam * b * lap / s
    assert np.max(np.abs(v - v_ref)) <= 1e-11 * np.max(np.abs(v_ref))


def test_vw_cosine_density_closed_form():
    Lx, Ly, Lz = 9.0, 7.0, 8.0
    g = Grid((Lx, Ly, Lz), (32, 16, 16))
    n0, eps, lam = 0.04, 0.2, 0.2
    # one period along x: the harmonics of sqrt(1 + eps cos) fall as
    # (eps / (1 + sqrt(1 - eps^2)))^m, 1e-16 at the Nyquist harmonic 16
    G = 2 * math.pi / Lx
    th = G * g.points()[..., 0]
    n = n0 * (1 + eps * np.cos(th))
    v, F = fn.vw_terms(g, n, lam)
    F_ref = lam / 8 * n0 * G * G * g.volume * (1 - math.sqrt(1 - eps * eps))
    assert abs(F - F_ref) <= 1e-12 * F_ref
    u = 1 + eps * np.cos(th)
    f2 = -0.5 * eps * G * G * np.cos(th) / np.sqrt(u) - 0.25 * (eps * G) ** 2 * np.sin(th) ** 2 / u ** 1.5
    v_ref = -0.5 * lam * f2 / np.sqrt(u)
    assert np.max(np.abs(v - v_ref)) <= 1e-12 * np.max(np.abs(v_ref))
    # second order in eps: lambda n0 eps^2 G^2 |Omega| / 16
    _, Fs = fn.vw_terms(g, n0 * (1 + 1e-4 * np.cos(th)), lam)
    assert abs(Fs - lam * n0 * 1e-8 * G * G * g.volume / 16) <= 1e-7 * Fs


def _one_center_case(A, B, sigma, tau):
    """One atom moved from r_old to r_new with the radial profile
    g(r) = A exp(-r^2/2 sigma^2) - B exp(-r^2/2 tau^2) + Ne/|Omega| (per cell):
    returns (system at r_new, its Ionic, prev spectra, brute-force raw density)."""
    L, N = 10.0, 40
    g = Grid((L, L, L), (N, N, N))
    Z = 3.0
    r_old, r_new = np.array([2.0, 3.0, 4.0]), np.array([6.1, 1.7, 5.3])
    s = scf.System(g.cell, g.shape, r_new[None], np.zeros(1, int), (Z,), (1.1,), (1.0,), W.ev(10.0), 0.2, True)
    n0 = s.Ne / g.volume

    def ghat(r0):  # Fourier coefficients of Z * profile (all k; aliasing below 1e-20)
        kr = g.k[0] * r0[0] + g.k[1] * r0[1] + g.k[2] * r0[2]
        prof = (A * (2 * math.pi * sigma ** 2) ** 1.5 * np.exp(-2 * math.pi ** 2 * sigma ** 2 * g.k2)
                - B * (2 * math.pi * tau ** 2) ** 1.5 * np.exp(-2 * math.pi ** 2 * tau ** 2 * g.k2))
        prof = np.where(g.k2 == 0, 0.0, prof)
        return Z * prof * np.exp(-2j * math.pi * kr)

    S_old = ionic.structure_factors(g, r_old[None], np.zeros(1, int), 1)[0]
    nhat_old = ghat(r_old)
    nhat_old[0, 0, 0] = s.Ne  # the k = 0 coefficient carries the N_e electrons
    raw = Z * _images(g, r_new, lambda d2: A * np.exp(-d2 / (2 * sigma ** 2)) - B * np.exp(-d2 / (2 * tau ** 2)))
    # the profile's own k = 0 part is removed above; add the mean back as the uniform part
    raw = raw - np.mean(raw) + n0
    return s, scf.ionic_setup(s), (nhat_old, Z * S_old), raw, n0


def test_one_center_floor_binds():
    # a shallow negative ring: the superposition dips below 1e-3 n0 over a few points,
    # and the floor adds far less than 1e-6 of the charge
    s, ion, prev, raw, n0 = _one_center_case(A=0.004, B=0.003824, sigma=0.8, tau=1.2)
    floor = scf.GUESS_FLOOR * n0
    assert np.min(raw) < floor  # the floor binds in this case
    added = s.grid.dv * float(np.sum(np.maximum(raw, floor) - raw))
    assert 0 < added <= scf.MAX_FLOOR_CHARGE * s.Ne
    n, fb = scf.initial_density(s, ion, "one_center", prev)
    assert not fb
    expect = np.maximum(raw, floor)
    expect *= s.Ne / (s.grid.dv * float(np.sum(expect)))
    assert np.max(np.abs(n - expect)) <= 1e-12 * np.max(expect)
    assert np.min(n) >= floor * (1 - 1e-6)
    assert abs(s.grid.integrate(n) - s.Ne) <= 1e-13 * s.Ne


def test_one_center_fallback_to_uniform():
    # a deep negative ring: the floor would add more than 1e-6 of the charge
    s, ion, prev, raw, n0 = _one_center_case(A=0.004, B=0.0040, sigma=0.8, tau=1.2)
    floor = scf.GUESS_FLOOR * n0
    added = s.grid.dv * float(np.sum(np.maximum(raw, floor) - raw))
    assert added > scf.MAX_FLOOR_CHARGE * s.Ne
    n, fb = scf.initial_density(s, ion, "one_center", prev)
    assert fb
    assert np.all(n == n0)
