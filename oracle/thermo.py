"""Oracle (test infrastructure only): free energy, pressure and forces at the
converged density, Sec. 2.6.

Free energy (Mermin functional of Sec. 2.2 at its stationary point):
  F = F_TF + F_vW + E_H + F_xc + E^ie + U^ii
  F_TF = int f0(n_a),  f0 = n kT eta - p0(eta)      (eta from the mu search)
The paper's internal energy replaces F_TF by K_e = (3/2) int p0 (Sec. 2.6.2);
vW and zero-T LDA carry no entropy.  The average-atom correction Delta E_AA is
not part of this path.

Pressure P = -(1/3) tr Sigma (Sec. 2.6), each trace written as the derivative
of the corresponding discrete energy under isotropic scaling of the cell at
fixed fractional coordinates and fixed grid counts:
  P_TF = (1/N_g) sum p0                         (Sec. 2.6.2, sigma^e)
  P_vW = 2 F_vW / (3 |Omega|)                   (F_vW scales as L^-2)
  P_H  = E_H / (3 |Omega|)                      (trace of sigma^ee, Sec. 2.6.4)
  P_xc = (1/N_g) sum n (v_xc - eps_xc)
  P_ie = E^ie/|Omega| + 1/(3|Omega|^2) Re sum_k conj(n^) |k| V^_s'(|k|) S_s  (Sec. 2.6.5)
  P_ii = U^ii / (3 |Omega|)   (alpha scales as 1/L, so U^ii scales as 1/L)
  P_kin = 2 K^i / (3 |Omega|) (Sec. 2.6.1; reported separately)
Forces F_j = F^ie_j + F^pm_j + F^pp_j (eq. force).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import fd
from . import functional as fn
from . import ionic
from .scf import Ionic, SCFResult, System


@dataclass
class Thermo:
    F: float
    E: float
    terms: dict
    P: float
    P_terms: dict
    forces: np.ndarray
    force_terms: dict


def evaluate(sys: System, ion: Ionic, res: SCFResult, forces=True, atoms=None) -> Thermo:
    g = sys.grid
    kT = sys.kT
    n = res.n
    eta = res.eta
    nhat = g.forward(n)
    p0 = fd.pressure0(eta, kT)
    F_TF = g.integrate(fd.density(eta, kT) * kT * eta - p0)
    K_e = 1.5 * g.integrate(p0)
    E_H = fn.hartree_energy(g, nhat)
    if sys.lam != 0.0:
        _, F_vW = fn.vw_terms(g, n, sys.lam)
    else:
        F_vW = 0.0
    if sys.xc:
        exc, vxc = fn.xc_terms(n)
        F_xc = g.integrate(n * exc)
        P_xc = float(np.sum(n * (vxc - exc))) / g.ng
    else:
        F_xc = 0.0
        P_xc = 0.0
    E_ie = ionic.electron_ion_energy(g, n, ion.Vie, sys.species, sys.Z, sys.rc)
    ew = ionic.ewald(g, sys.pos, sys.Zj, ion.SZ, alpha=sys.ewald_alpha if sys.ewald_alpha > 0 else None,
                     atoms=atoms if forces else [])
    U_ii = ew["U_ii"]
    F = F_TF + F_vW + E_H + F_xc + E_ie + U_ii
    E = K_e + F_vW + E_H + F_xc + E_ie + U_ii
    P_TF = float(np.sum(p0)) / g.ng
    P_vW = 2.0 * F_vW / (3.0 * g.volume)
    P_H = E_H / (3.0 * g.volume)
    P_ie = ionic.electron_ion_pressure(g, nhat, ion.S, E_ie, sys.Z, sys.rc)
    P_ii = U_ii / (3.0 * g.volume)
    P = P_TF + P_vW + P_H + P_xc + P_ie + P_ii
    terms = dict(F_TF=F_TF, K_e=K_e, F_vW=F_vW, E_H=E_H, F_xc=F_xc, E_ie=E_ie, U_ii=U_ii,
                 U_pp=ew["U_pp"], U_pm=ew["U_pm"], U_je=ew["U_je"], alpha=ew["alpha"])
    P_terms = dict(P_TF=P_TF, P_vW=P_vW, P_H=P_H, P_xc=P_xc, P_ie=P_ie, P_ii=P_ii)
    if forces:
        sel = list(range(sys.pos.shape[0])) if atoms is None else list(atoms)
        F_ie = ionic.electron_ion_forces(g, nhat, sys.pos, sys.species, sys.Z, sys.rc, sel)
        F_pm = ew["F_pm"][sel]
        F_pp = ew["F_pp"][sel]
        Ftot = F_ie + F_pm + F_pp
        fterms = dict(F_ie=F_ie, F_pm=F_pm, F_pp=F_pp)
    else:
        Ftot = None
        fterms = {}
    return Thermo(F, E, terms, P, P_terms, Ftot, fterms)


def ion_kinetic(sys: System, vel) -> float:
    m = np.array([sys.mass[s] for s in sys.species])
    return 0.5 * float(np.sum(m[:, None] * np.asarray(vel) ** 2))


def ion_kinetic_pressure(sys: System, vel) -> float:
    return 2.0 * ion_kinetic(sys, vel) / (3.0 * sys.grid.volume)
