"""Pins for the oracle's transforms, Hartree term, LDA, Ewald sum and Verlet
step against closed forms, brute-force sums and textbook constants."""
import math

import numpy as np
import pytest
from scipy.special import erfc

from oracle import functional as fn
from oracle import ionic, md
from oracle.grid import Grid


def periodic_gaussian(g: Grid, center, sigma, Q=1.0, images=2):
    X = g.points()
    rho = np.zeros(g.shape)
    L = np.array(g.cell)
    for i in range(-images, images + 1):
        for j in range(-images, images + 1):
            for k in range(-images, images + 1):
                d = X - (np.asarray(center) + L * np.array([i, j, k]))
                rho += np.exp(-np.sum(d * d, axis=-1) / (2 * sigma ** 2))
    return Q * rho / (2 * math.pi * sigma ** 2) ** 1.5


def test_transform_of_gaussian_and_roundtrip():
    g = Grid((9.0, 10.0, 11.0), (24, 24, 28))
    sigma = 3.2 * max(L / n for L, n in zip(g.cell, g.shape))
    c = np.array([1.3, 2.9, 7.4])
    rho = periodic_gaussian(g, c, sigma)
    F = g.forward(rho)
    kc = g.k[0] * c[0] + g.k[1] * c[1] + g.k[2] * c[2]
    ref = np.exp(-2 * math.pi ** 2 * sigma ** 2 * g.k2) * np.exp(-2j * math.pi * kc)
    assert np.max(np.abs(F - ref)) <= 1e-12
    assert np.max(np.abs(g.inverse(F) - rho)) <= 1e-12 * rho.max()
    assert abs(g.integrate(rho) - 1.0) <= 1e-13


def test_hartree_energy_of_gaussian():
    g = Grid((12.0, 12.0, 12.0), (32, 32, 32))
    sigma = 3.0 * 12.0 / 32
    Q = 2.5
    rho = periodic_gaussian(g, (3.0, 4.0, 5.0), sigma, Q)
    E = fn.hartree_energy(g, g.forward(rho))
    # analytic lattice sum over all k (beyond the box), neutralising background
    m = np.arange(-40, 41)
    MX, MY, MZ = np.meshgrid(m, m, m, indexing="ij")
    k2 = (MX ** 2 + MY ** 2 + MZ ** 2) / 12.0 ** 2
    k2 = k2[k2 > 0]
    ref = Q * Q / (2 * math.pi * g.volume) * np.sum(np.exp(-4 * math.pi ** 2 * sigma ** 2 * k2) / k2)
    assert abs(E - ref) <= 1e-12 * abs(ref)
    # Poisson: lap V_H = -4 pi (rho - <rho>), checked spectrally-independent by finite differences
    V = fn.hartree_potential(g, g.forward(rho))
    h = 12.0 / 32
    lap = sum(np.roll(V, 1, a) + np.roll(V, -1, a) - 2 * V for a in range(3)) / h ** 2
    src = -4 * math.pi * (rho - rho.mean())
    assert np.max(np.abs(lap - src)) <= 2e-2 * np.max(np.abs(src))  # O(h^2) stencil error


def test_lda_pz81_derivative_and_continuity():
    n = np.array([1e-4, 3e-3, 0.02, 0.1, 0.5, 3.0])
    h = 1e-6
    e_p = (n * (1 + h)) * fn.eps_c(n * (1 + h))
    e_m = (n * (1 - h)) * fn.eps_c(n * (1 - h))
    vnum = (e_p - e_m) / (2 * h * n)
    assert np.max(np.abs(vnum - fn.v_c(n)) / np.abs(fn.v_c(n))) <= 1e-8
    ex_p = (n * (1 + h)) * fn.eps_x(n * (1 + h))
    ex_m = (n * (1 - h)) * fn.eps_x(n * (1 - h))
    assert np.max(np.abs((ex_p - ex_m) / (2 * h * n) - fn.v_x(n)) / np.abs(fn.v_x(n))) <= 1e-8
    # the two PZ81 branches meet at r_s = 1 (to the 4 digits of the published constants)
    n1 = 3.0 / (4.0 * math.pi)
    hi = -0.1423 / (1 + 1.0529 + 0.3334)
    lo = 0.0311 * 0.0 - 0.048 + 0.0 - 0.0116
    assert abs(hi - lo) <= 1e-4
    assert abs(fn.eps_c(np.array([n1 * (1 + 1e-12)]))[0] - fn.eps_c(np.array([n1 * (1 - 1e-12)]))[0]) <= 1e-4
    # Dirac exchange in closed form: eps_x = -(3/4)(3/pi)^(1/3) n^(1/3)
    assert abs(fn.eps_x(np.array([1.0]))[0] + 0.75 * (3 / math.pi) ** (1 / 3)) <= 1e-15


def fcc_lattice(cells, L):
    a = L / cells
    b = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    return np.array([(np.array([i, j, k]) + x) * a for i in range(cells) for j in range(cells)
                     for k in range(cells) for x in b])


def brute_ewald(pos, Z, L, alpha, nimg=3, mmax=12):
    """Independent Ewald energy: explicit image sum in real space, explicit k-sum."""
    n = len(pos)
    U = 0.0
    shifts = [np.array([i, j, k]) * L for i in range(-nimg, nimg + 1) for j in range(-nimg, nimg + 1)
              for k in range(-nimg, nimg + 1)]
    for a in range(n):
        for b in range(n):
            for s in shifts:
                d = pos[a] - pos[b] + s
                r = math.sqrt(d @ d)
                if r > 0:
                    U += 0.5 * Z * Z * erfc(alpha * r) / r
    V = L ** 3
    m = np.arange(-mmax, mmax + 1)
    for mx in m:
        for my in m:
            for mz in m:
                if mx == my == mz == 0:
                    continue
                k = np.array([mx, my, mz]) / L
                k2 = k @ k
                S = np.sum(Z * np.exp(-2j * math.pi * pos @ k))
                U += 0.5 / V * math.exp(-math.pi ** 2 * k2 / alpha ** 2) / (math.pi * k2) * abs(S) ** 2
    U -= alpha / math.sqrt(math.pi) * n * Z * Z
    U -= math.pi * (n * Z) ** 2 / (2 * alpha ** 2 * V)
    return U


def test_ewald_fcc_madelung():
    L = 15.302634575373462
    pos = fcc_lattice(2, L)
    Z = 3.0
    g = Grid((L, L, L), (64, 64, 64))
    S = ionic.structure_factors(g, pos, np.zeros(32, dtype=int), 1)
    ew = ionic.ewald(g, pos, np.full(32, Z), Z * S[0])
    rws = (3 * L ** 3 / (4 * math.pi * 32)) ** (1 / 3)
    # textbook fcc Madelung energy in the Wigner-Seitz convention
    assert abs(ew["U_ii"] / 32 / (Z * Z / rws) + 0.8958736) <= 2e-7
    ref = brute_ewald(pos[:], Z, L, alpha=0.35, nimg=2, mmax=8)
    assert abs(ew["U_ii"] - ref) <= 1e-10 * abs(ref)
    assert np.max(np.abs(ew["F_pp"] + ew["F_pm"])) <= 1e-12  # perfect lattice: no force


def test_ewald_alpha_independence_and_momentum():
    rng = np.random.default_rng(7)
    L = 11.0
    pos = rng.uniform(0, L, (6, 3))
    Zj = np.array([3.0, 3.0, 3.0, 1.0, 1.0, 2.0])
    sp = np.array([0, 0, 0, 1, 1, 2])
    # both truncation errors fall as exp(-pi N / 4) at the balanced alpha
    for N, fac, tol in ((32, 0.92, 1e-9), (64, 1.2, 1e-11), (64, 0.8, 1e-11)):
        g = Grid((L, L, L), (N, N, N))
        S = ionic.structure_factors(g, pos, sp, 3)
        SZ = ionic.charge_structure_factor(S, (3.0, 1.0, 2.0))
        a0 = ionic.ewald_alpha(g)
        e0 = ionic.ewald(g, pos, Zj, SZ, a0)
        e1 = ionic.ewald(g, pos, Zj, SZ, fac * a0)
        assert abs(e0["U_ii"] - e1["U_ii"]) <= tol * abs(e0["U_ii"])
        assert np.max(np.abs(e0["F_pp"] + e0["F_pm"] - e1["F_pp"] - e1["F_pm"])) <= 1e3 * tol
        assert np.max(np.abs(e0["F_pp"].sum(0))) <= 1e-12
        assert np.max(np.abs(e0["F_pm"].sum(0))) <= 1e-12
    # ion-ion forces are minus the gradient of U_ii (central differences)
    g = Grid((L, L, L), (64, 64, 64))
    base = ionic.ewald(g, pos, Zj, ionic.charge_structure_factor(ionic.structure_factors(g, pos, sp, 3), (3.0, 1.0, 2.0)))
    h = 1e-5
    for a in range(3):
        p = pos.copy(); p[2, a] += h
        m = pos.copy(); m[2, a] -= h
        up = ionic.ewald(g, p, Zj, ionic.charge_structure_factor(ionic.structure_factors(g, p, sp, 3), (3.0, 1.0, 2.0)))["U_ii"]
        um = ionic.ewald(g, m, Zj, ionic.charge_structure_factor(ionic.structure_factors(g, m, sp, 3), (3.0, 1.0, 2.0)))["U_ii"]
        f = base["F_pp"][2, a] + base["F_pm"][2, a]
        assert abs(-(up - um) / (2 * h) - f) <= 1e-7 * max(1.0, abs(f))
    # printed stress-tensor trace agrees with the scaling form U_ii/(3|Omega|)
    p_tr = ionic.ewald_stress_trace_printed(g, pos, Zj, ionic.charge_structure_factor(
        ionic.structure_factors(g, pos, sp, 3), (3.0, 1.0, 2.0)), base["alpha"])
    assert abs(p_tr - base["U_ii"] / (3 * L ** 3)) <= 1e-10 * abs(base["U_ii"] / L ** 3)


def test_form_factor_coulomb_limit_and_derivative():
    g = Grid((10.0, 10.0, 10.0), (16, 16, 16))
    V0 = ionic.form_factor(g, 3.0, 0.0)
    nz = g.nonzero
    assert np.allclose(V0[nz], -3.0 / (math.pi * g.k2[nz]), rtol=1e-15, atol=0)
    h = 1e-6
    q = np.array([0.13, 0.7, 1.9])
    Vs = lambda qq: -3.0 * np.cos(2 * math.pi * qq * 1.1) / (math.pi * qq * qq)
    g2 = Grid((1.0, 1.0, 1.0), (2, 2, 2))
    # derivative formula against central differences
    for qq in q:
        num = (Vs(qq + h) - Vs(qq - h)) / (2 * h)
        a = 2 * math.pi * qq * 1.1
        ana = 3.0 * (2 * math.pi * 1.1 * math.sin(a) / qq ** 2 + 2 * math.cos(a) / qq ** 3) / math.pi
        assert abs(num - ana) <= 1e-7 * abs(ana)
    # E_alpha is the k->0 limit of V_s + Z/(pi k^2) = 2 pi Z rc^2
    qq = 1e-5
    assert abs((Vs(qq) + 3.0 / (math.pi * qq * qq)) - 2 * math.pi * 3.0 * 1.1 ** 2) <= 1e-5


def test_verlet_free_particle_and_reversibility():
    m = np.array([2.0, 5.0])
    r0 = np.array([[0.1, 0.2, 0.3], [1.0, -1.0, 0.5]])
    v0 = np.array([[0.01, -0.02, 0.03], [0.0, 0.04, -0.01]])
    dt = 0.7
    F0 = np.zeros_like(r0)
    rp = md.verlet_start(r0, v0, F0, m, dt)
    r, rprev = r0, rp
    for s in range(10):
        rn, v = md.verlet_step(r, rprev, F0, m, dt)
        assert np.allclose(v, v0, rtol=0, atol=1e-15)
        rprev, r = r, rn
    assert np.allclose(r, r0 + 10 * dt * v0, rtol=0, atol=1e-13)
    # constant force: exact parabola; time reversal returns to start
    F = np.array([[0.3, 0.0, -0.2], [0.1, 0.1, 0.1]])
    rp = md.verlet_start(r0, v0, F, m, dt)
    r, rprev = r0, rp
    for s in range(5):
        rn, v = md.verlet_step(r, rprev, F, m, dt)
        rprev, r = r, rn
    t = 5 * dt
    assert np.allclose(r, r0 + v0 * t + 0.5 * F / m[:, None] * t * t, rtol=0, atol=1e-12)
    r, rprev = rprev, r  # reverse
    for s in range(4):
        rn, v = md.verlet_step(r, rprev, F, m, dt)
        rprev, r = r, rn
    assert np.allclose(r, r0, rtol=0, atol=1e-12)
