"""Pins for the oracle's Fermi-Dirac integrals and Thomas-Fermi relations.

Independent references: mpmath's polylog identity
I_j(x) = -Gamma(j+1) Li_{j+1}(-e^x), the closed form at x = 0
(Gamma(j+1)(1-2^{-j})zeta(j+1)), the non-degenerate series, the Sommerfeld
expansion, and the derivative identity dI_j/dx = j I_{j-1}.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.special import gamma, zeta

from oracle import fd

ORDERS = (("m12", -0.5), ("p12", 0.5), ("p32", 1.5))


def mp_fd(j, x):
    with mp.workdps(30):
        return float(mp.re(-mp.gamma(j + 1) * mp.polylog(j + 1, -mp.exp(mp.mpf(float(x))))))


def test_fd_vs_mpmath_polylog_random():
    rng = np.random.default_rng(1234)
    xs = np.concatenate([rng.uniform(-100.0, 1000.0, 350), rng.uniform(-10.0, 60.0, 350),
                         np.array([-100.0, -40.0, -1e-3, 0.0, 1e-3, 40.0, 45.0, 85.0, 1000.0])])
    v = fd.fd_integrals(xs)
    for name, j in ORDERS:
        ref = np.array([mp_fd(j, x) for x in xs])
        rel = np.abs(v[name] - ref) / np.abs(ref)
        assert rel.max() <= 1e-14, (name, xs[np.argmax(rel)], rel.max())


@pytest.mark.parametrize("name,j", ORDERS)
def test_fd_at_zero_closed_form(name, j):
    ref = gamma(j + 1) * (1.0 - 2.0 ** (-j)) * zeta(j + 1)
    got = fd.fd_integrals(np.array([0.0]))[name][0]
    assert abs(got - ref) <= 2e-15 * abs(ref)


@pytest.mark.parametrize("name,j", ORDERS)
def test_fd_nondegenerate_series(name, j):
    xs = np.array([-3.0, -7.5, -20.0, -60.0])
    got = fd.fd_integrals(xs)[name]
    for x, g in zip(xs, got):
        s = sum((-1) ** (k + 1) * math.exp(k * x) / k ** (j + 1) for k in range(1, 80))
        ref = gamma(j + 1) * s
        assert abs(g - ref) <= 1e-14 * abs(ref)


@pytest.mark.parametrize("name,j", ORDERS)
def test_fd_sommerfeld(name, j):
    # I_j(x) ~ x^{j+1}/(j+1) [1 + sum_k 2(1-2^{1-2k}) zeta(2k) (j+1)j...(j+2-2k) x^{-2k}]
    for x in (60.0, 150.0, 900.0):
        acc = 1.0
        for k in range(1, 8):
            c = 2.0 * (1.0 - 2.0 ** (1 - 2 * k)) * zeta(2 * k)
            for i in range(2 * k):
                c *= (j + 1 - i)
            acc += c * x ** (-2 * k)
        ref = x ** (j + 1) / (j + 1) * acc
        got = fd.fd_integrals(np.array([x]))[name][0]
        assert abs(got - ref) <= 2e-15 * abs(ref), (x, got, ref)


def test_fd_derivative_identity():
    xs = np.array([-5.0, -0.3, 0.7, 3.0, 12.0, 40.0])
    h = 1e-3
    # 4th-order central difference of I_{1/2} and I_{3/2}
    def d(name, x):
        f = lambda t: fd.fd_integrals(np.array([t]))[name][0]
        return (-f(x + 2 * h) + 8 * f(x + h) - 8 * f(x - h) + f(x - 2 * h)) / (12 * h)
    for x in xs:
        v = fd.fd_integrals(np.array([x]))
        assert abs(d("p12", x) - 0.5 * v["m12"][0]) <= 1e-10 * abs(v["m12"][0])
        assert abs(d("p32", x) - 1.5 * v["p12"][0]) <= 1e-10 * abs(v["p12"][0])


def test_fd_inverse_roundtrip():
    for x in (-30.0, -2.0, 0.0, 0.2760068207, 1.9, 11.5873, 300.0):
        y = fd.I_p12(np.array([x]))[0]
        assert abs(fd.I_p12_inverse(y) - x) <= 1e-13 * max(1.0, abs(x))


# ---- ideal Fermi gas closed forms ----
N0_AL = 3.0 / (15.302634575373462 ** 3 / 32.0)  # electrons per bohr^3 at 2.7 g/cm^3


@pytest.mark.parametrize("T_ev", [1.0, 5.0, 10.0])
def test_uniform_gas_vs_mpmath(T_ev):
    kT = T_ev / 27.211386245988
    eta = fd.I_p12_inverse(N0_AL / fd.c_n(kT))
    with mp.workdps(30):
        cn = (2 * mp.mpf(kT)) ** 1.5 / (2 * mp.pi ** 2)
        f = lambda e: mp.re(-mp.gamma(1.5) * mp.polylog(1.5, -mp.exp(e))) * cn - N0_AL
        eta_ref = mp.re(mp.findroot(f, eta))
        p_ref = (2 * mp.sqrt(2) / (3 * mp.pi ** 2)) * mp.mpf(kT) ** 2.5 * \
            mp.re(-mp.gamma(2.5) * mp.polylog(2.5, -mp.exp(eta_ref)))
    assert abs(eta - float(eta_ref)) <= 1e-12 * max(1.0, abs(float(eta_ref)))
    p = fd.pressure0(np.array([eta]), kT)[0]
    assert abs(p - float(p_ref)) <= 1e-13 * float(p_ref)


def test_degenerate_and_classical_limits():
    n0 = N0_AL
    kT = 1e-5
    eta = fd.I_p12_inverse(n0 / fd.c_n(kT))
    EF = (3 * math.pi ** 2 * n0) ** (2.0 / 3.0) / 2.0
    p = fd.pressure0(np.array([eta]), kT)[0]
    # Sommerfeld: P = (2/5) n EF [1 + (5 pi^2/12)(kT/EF)^2]
    assert abs(p - 0.4 * n0 * EF * (1 + 5 * math.pi ** 2 / 12 * (kT / EF) ** 2)) <= 1e-9 * p
    assert abs(kT * eta - EF * (1 - math.pi ** 2 / 12 * (kT / EF) ** 2)) <= 1e-9 * EF
    kT = 50.0
    eta = fd.I_p12_inverse(n0 / fd.c_n(kT))
    p = fd.pressure0(np.array([eta]), kT)[0]
    # P = n kT (1 + n lambda^3 / 2^{7/2} + ...), thermal wavelength lambda = sqrt(2 pi / kT),
    # spin degeneracy 2 (first quantum correction of the ideal Fermi gas)
    lam3 = (2 * math.pi / kT) ** 1.5
    assert abs(p - n0 * kT * (1 + n0 * lam3 / 2 ** 3.5)) <= 1e-8 * p


def test_free_energy_density_derivative():
    # df0/dn = kT eta(n)
    for T_ev in (1.0, 10.0):
        kT = T_ev / 27.211386245988
        eta = np.array([-2.0, 0.3, 4.0, 15.0])
        n = fd.density(eta, kT)
        h = 1e-6
        for e, nn in zip(eta, n):
            ep = fd.I_p12_inverse(nn * (1 + h) / fd.c_n(kT))
            em = fd.I_p12_inverse(nn * (1 - h) / fd.c_n(kT))
            fp = fd.free_energy_density0(np.array([ep]), kT)[0]
            fm = fd.free_energy_density0(np.array([em]), kT)[0]
            assert abs((fp - fm) / (2 * h * nn) - kT * e) <= 1e-7 * max(1.0, abs(kT * e))


def test_inverse_array_round_trip_and_scalar_agreement():
    y = np.logspace(-30, 6, 73)
    x = fd.I_p12_inverse_array(y)
    back = fd.I_p12(x)
    assert np.max(np.abs(back - y) / y) <= 1e-13
    for k in (0, 20, 40, 60, 72):
        assert abs(x[k] - fd.I_p12_inverse(float(y[k]))) <= 1e-12 * max(1.0, abs(x[k]))
    # the brackets hold the root, and a start anywhere converges to the same X
    lo = np.log(y / math.gamma(1.5))
    hi = np.maximum((1.5 * y) ** (2.0 / 3.0), lo + 1.0) + 1.0
    assert np.all(fd.I_p12(lo - 1e-9) < y) and np.all(fd.I_p12(hi) > y)
    x2 = fd.I_p12_inverse_array(y, x + np.linspace(-30.0, 30.0, y.size))
    assert np.max(np.abs(x2 - x) / np.maximum(1.0, np.abs(x))) <= 1e-14


def test_secant_K_reduces_to_the_second_order_form():
    """K = int kT (eta(n_i) - eta_a) dn equals int dn^2 / (dn_a/dmu) to second order in dn."""
    rng = np.random.default_rng(3)
    kT = 0.2
    cn = fd.c_n(kT)
    eta_a = rng.uniform(-5.0, 20.0, 400)
    n_a = cn * fd.I_p12(eta_a)
    chi = cn / (2.0 * kT) * fd.I_m12(eta_a)
    shape = rng.normal(size=400)
    ratios = []
    for eps in (1e-2, 1e-3, 1e-4):
        dn = eps * n_a * shape
        eta_i = fd.I_p12_inverse_array((n_a + dn) / cn)
        Ks = np.sum(kT * (eta_i - eta_a) * dn)
        Kc = np.sum(dn * dn / chi)
        ratios.append(abs(Ks / Kc - 1.0))
    assert ratios[0] < 0.05 and ratios[1] < ratios[0] / 5 and ratios[2] < ratios[1] / 5
