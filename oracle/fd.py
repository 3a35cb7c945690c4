"""Oracle (test infrastructure only): complete Fermi-Dirac integrals and the
local Thomas-Fermi relations built on them.

Paper, Sec. 2.2 (equation SCF1): the finite-temperature Thomas-Fermi density is
    n = (2 kT)^{3/2} / (2 pi^2) * I_{1/2}((mu - V)/kT),
with I_j(x) = int_0^inf t^j / (exp(t - x) + 1) dt.
Sec. 2.6.2 gives the electron kinetic energy K_e = kT int c_TF I_{3/2}(eta),
c_TF = sqrt(2)/pi^2 (kT)^{3/2}, and the stress -2 K_e / (3 |Omega|).
Sec. 2.4 names the inverse I_{1/2}^{-1} used to invert SCF1.

The integrals come from the plain-C quadrature of the definition in
``fd_quad.c``; nothing here approximates them otherwise.
"""
from __future__ import annotations

import math

import numpy as np

from . import _native

# 16-point Gauss-Legendre rule per panel (library primitive for the nodes).
_GX, _GW = np.polynomial.legendre.leggauss(16)
_GX = np.ascontiguousarray(_GX, dtype=np.float64)
_GW = np.ascontiguousarray(_GW, dtype=np.float64)


def fd_integrals(x, orders=("m12", "p12", "p32")):
    """Return a dict {order: I_j(x)} for j = -1/2 ('m12'), 1/2 ('p12'), 3/2 ('p32')."""
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    flat = xa.reshape(-1)
    out = {k: (np.empty_like(flat) if k in orders else None) for k in ("m12", "p12", "p32")}
    _native.lib().oracle_fd_eval(flat.size, _native.as_ptr(flat), _GX.size, _native.as_ptr(_GX),
                                 _native.as_ptr(_GW), _native.as_ptr(out["m12"]),
                                 _native.as_ptr(out["p12"]), _native.as_ptr(out["p32"]))
    return {k: out[k].reshape(xa.shape) for k in orders}


def I_m12(x):
    return fd_integrals(x, ("m12",))["m12"]


def I_p12(x):
    return fd_integrals(x, ("p12",))["p12"]


def I_p32(x):
    return fd_integrals(x, ("p32",))["p32"]


def I_p12_inverse_array(y, x0=None):
    """Element-wise X(y) with I_{1/2}(X) = y for an array y > 0: Newton
    safeguarded by bisection inside the bracket lo = ln(y / Gamma(3/2))
    (I_{1/2}(x) < Gamma(3/2) e^x) and hi = max((3y/2)^{2/3}, lo + 1) + 1
    (I_{1/2}(x) > x^{3/2} / (3/2) for x > 0), started from x0 when given."""
    y = np.asarray(y, dtype=np.float64)
    if not np.all(y > 0.0):
        raise ValueError("I_{1/2}^{-1} needs y > 0")
    lo = np.log(y / math.gamma(1.5)) - 1e-9
    hi = np.maximum((1.5 * y) ** (2.0 / 3.0), lo + 1.0) + 1.0
    x = 0.5 * (lo + hi) if x0 is None else np.clip(np.asarray(x0, dtype=np.float64), lo, hi)
    x = np.array(x, dtype=np.float64).reshape(y.shape)
    lo = np.broadcast_to(lo, y.shape).copy()
    hi = np.broadcast_to(hi, y.shape).copy()
    # each element iterates on its own; only the unfinished ones are evaluated
    act = np.flatnonzero(np.ones(y.shape, dtype=bool))
    xf, lof, hif, yf = x.reshape(-1), lo.reshape(-1), hi.reshape(-1), y.reshape(-1)
    for _ in range(200):
        xa = xf[act]
        v = fd_integrals(xa, ("m12", "p12"))
        f = v["p12"] - yf[act]
        hia = np.where(f > 0, xa, hif[act])
        loa = np.where(f <= 0, xa, lof[act])
        xn = xa - f / (0.5 * v["m12"])
        xn = np.where((loa < xn) & (xn < hia), xn, 0.5 * (loa + hia))
        fin = np.abs(xn - xa) <= 2e-16 * np.maximum(1.0, np.abs(xa))
        xf[act], lof[act], hif[act] = xn, loa, hia
        act = act[~fin]
        if act.size == 0:
            return x
    raise RuntimeError("I_{1/2}^{-1} did not converge")


def I_p12_inverse(y: float) -> float:
    """X(y) with I_{1/2}(X) = y, y > 0 (Sec. 2.4).  Safeguarded Newton on the
    monotone I_{1/2}, derivative dI_{1/2}/dx = (1/2) I_{-1/2}."""
    if not (y > 0.0):
        raise ValueError("I_{1/2}^{-1} needs y > 0")
    # bracket: I_{1/2}(x) < Gamma(3/2) e^x for all x and I_{1/2}(x) > x^{3/2}/(3/2) for x > 0
    lo = math.log(y / math.gamma(1.5)) - 1e-9
    hi = max((1.5 * y) ** (2.0 / 3.0), lo + 1.0) + 1.0
    while I_p12(np.array([hi]))[0] < y:
        hi = 2.0 * hi + 1.0
    while I_p12(np.array([lo]))[0] > y:
        lo = lo - 1.0
    x = 0.5 * (lo + hi)
    for _ in range(200):
        v = fd_integrals(np.array([x]), ("m12", "p12"))
        f = v["p12"][0] - y
        if f > 0:
            hi = x
        else:
            lo = x
        d = 0.5 * v["m12"][0]
        xn = x - f / d
        if not (lo < xn < hi):
            xn = 0.5 * (lo + hi)
        if abs(xn - x) <= 2e-16 * max(1.0, abs(x)):
            x = xn
            break
        x = xn
    return float(x)


# ---- local Thomas-Fermi relations (Sec. 2.2 SCF1, Sec. 2.6.2) ----

def c_n(kT: float) -> float:
    """n = c_n I_{1/2}(eta), c_n = (2 kT)^{3/2} / (2 pi^2)."""
    return (2.0 * kT) ** 1.5 / (2.0 * math.pi ** 2)


def density(eta, kT):
    return c_n(kT) * I_p12(eta)


def ddensity_dmu(eta, kT):
    """dn/dmu = c_n / kT * dI_{1/2}/deta = c_n / (2 kT) I_{-1/2}(eta)."""
    return c_n(kT) / (2.0 * kT) * I_m12(eta)


def pressure0(eta, kT):
    """Ideal Fermi-gas pressure p0 = (2/3) x kinetic-energy density
    = (2/3) kT c_TF I_{3/2}(eta) with c_TF = sqrt(2)/pi^2 (kT)^{3/2}."""
    return (2.0 / 3.0) * kT * (math.sqrt(2.0) / math.pi ** 2) * kT ** 1.5 * I_p32(eta)


def free_energy_density0(eta, kT):
    """f0 at the density n(eta): f0 = n kT eta - p0 (Legendre transform of p0;
    the paper's sigma^e identity f0 - n df0/dn = -p0)."""
    return density(eta, kT) * kT * np.asarray(eta) - pressure0(eta, kT)
