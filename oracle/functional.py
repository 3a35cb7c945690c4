"""Oracle (test infrastructure only): the density functional terms beyond
Thomas-Fermi, on the grid of ``oracle.grid``.

Hartree (Sec. 2.3, Poisson solution; Sec. 2.6.4 discrete energy):
    V^_H(k) = n^(k) / (pi |k|^2), V^_H(0) = 0
    E_H = 1/(2|Omega|) sum_{k != 0} |n^(k)|^2 / (pi |k|^2)

von Weizsaecker (Sec. 2.2 names the gradient correction; its form is not
printed).  Standard form with s = sqrt(n):
    F_vW = (lambda/8) int |grad n|^2 / n = (lambda/2) int |grad s|^2
         = (lambda/2) (1/|Omega|) sum_k (2 pi |k|)^2 |s^(k)|^2
    v_vW = dF_vW/dn = -(lambda/2) (lap s) / s,  lap s = inverse(-(2 pi |k|)^2 s^)

LDA exchange-correlation (the paper uses libxc's zero-temperature LDA; the
specific functional is not named).  Reading: Dirac exchange plus the
Perdew-Zunger 1981 parametrisation of the unpolarised correlation energy.
    eps_x = -(3/4) (3 n / pi)^{1/3},   v_x = (4/3) eps_x
    r_s >= 1: eps_c = g / (1 + b1 sqrt(r_s) + b2 r_s)
    r_s <  1: eps_c = A ln r_s + B + C r_s ln r_s + D r_s
    v_c = eps_c - (r_s/3) d eps_c / d r_s
Parity of the PZ81 constants themselves is unpinned (the publication is not
available); the code is pinned by finite differences of n*eps_xc and by the
continuity of the two branches at r_s = 1.
"""
from __future__ import annotations

import math

import numpy as np

from .grid import Grid

PZ_GAMMA, PZ_B1, PZ_B2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116


# ---------------- Hartree ----------------
def hartree_kernel(g: Grid) -> np.ndarray:
    K = np.zeros(g.shape)
    K[g.nonzero] = 1.0 / (math.pi * g.k2[g.nonzero])
    return K


def hartree_potential(g: Grid, nhat: np.ndarray) -> np.ndarray:
    return g.inverse(nhat * hartree_kernel(g))


def hartree_energy(g: Grid, nhat: np.ndarray) -> float:
    return 0.5 * g.box_sum(np.abs(nhat) ** 2 * hartree_kernel(g))


# ---------------- von Weizsaecker ----------------
def vw_terms(g: Grid, n: np.ndarray, lam: float):
    """Return (v_vW(r), F_vW) for density n."""
    s = np.sqrt(n)
    shat = g.forward(s)
    q2 = (2.0 * math.pi) ** 2 * g.k2
    lap = g.inverse(-q2 * shat)
    v = -0.5 * lam * lap / s
    F = 0.5 * lam * g.box_sum(q2 * np.abs(shat) ** 2)
    return v, F


# ---------------- LDA xc ----------------
def rs_of(n):
    return (3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)


def eps_x(n):
    return -0.75 * (3.0 * n / math.pi) ** (1.0 / 3.0)


def v_x(n):
    return (4.0 / 3.0) * eps_x(n)


def eps_c(n):
    rs = rs_of(np.asarray(n, dtype=np.float64))
    hi = PZ_GAMMA / (1.0 + PZ_B1 * np.sqrt(rs) + PZ_B2 * rs)
    with np.errstate(divide="ignore", invalid="ignore"):
        lo = PZ_A * np.log(rs) + PZ_B + PZ_C * rs * np.log(rs) + PZ_D * rs
    return np.where(rs >= 1.0, hi, lo)


def deps_c_drs(n):
    rs = rs_of(np.asarray(n, dtype=np.float64))
    den = 1.0 + PZ_B1 * np.sqrt(rs) + PZ_B2 * rs
    hi = -PZ_GAMMA * (0.5 * PZ_B1 / np.sqrt(rs) + PZ_B2) / den ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        lo = PZ_A / rs + PZ_C * np.log(rs) + PZ_C + PZ_D
    return np.where(rs >= 1.0, hi, lo)


def v_c(n):
    rs = rs_of(np.asarray(n, dtype=np.float64))
    return eps_c(n) - rs / 3.0 * deps_c_drs(n)


def xc_terms(n):
    """Return (eps_xc(r), v_xc(r)) pointwise."""
    return eps_x(n) + eps_c(n), v_x(n) + v_c(n)
