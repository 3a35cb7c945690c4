"""Oracle (test infrastructure only): everything that depends on the ion
positions -- structure factor, local pseudopotential field, Ewald ion-ion
energy and forces, electron-ion energy, forces and pressure term.

Structure factor (Sec. 2.4):  S_s(k) = sum_{j in s} exp(-2 pi i k.r_j)
Charge-weighted (Sec. 2.5.1): S_Z = sum_s Z_s S_s
Ionic field (Sec. 2.4, eq. iepseudo, with V^_s(0) = 0 per Payne):
    V^ie^(k) = sum_s V^_s(k) S_s(k)
Form factor (empty-core local pseudopotential, fixed by the workload):
    V^_s(k) = -Z_s cos(2 pi |k| r_c) / (pi |k|^2)    [= -4 pi Z cos(G r_c)/G^2]
  or tabulated (eq. iepseudo takes any radial local pseudopotential): the
  non-Coulomb part D_s(q) = V^_s(q) + Z_s/(pi q^2), q = |k|, given at the nodes
  q_i = i dq, and between nodes the cubic through the four nodes i-1, i, i+1,
  i+2 around q (Lagrange interpolation; D_s is even in q, so node -1 carries
  the value of node 1).  dV^_s/dq is that cubic's derivative plus
  2 Z_s/(pi q^3); D_s(0) is the k = 0 limit entering E_alpha.
Ewald (Sec. 2.6.3): U^ii = U^pp + U^pm + U^je with
    U^pp = sum_{j<l} Z_j Z_l erfc(alpha d)/d         (minimum image)
    U^pm = 1/(2|Omega|) sum_{k != 0} V^_alpha |S_Z|^2 - alpha/sqrt(pi) sum_j Z_j^2
    V^_alpha = exp(-(pi k/alpha)^2) / (pi k^2)
    U^je = -pi Q^2 / (2 alpha^2 |Omega|)
    F^pp_j = sum_{l != j} Z_j Z_l [erfc(alpha d)/d + 2 alpha/sqrt(pi) exp(-alpha^2 d^2)] d_vec/d^2,
             d_vec = r_j - r_l (minimum image; repulsive)
    F^pm_j = Z_j (2 pi/|Omega|) sum_{k != 0} V^_alpha Im(exp(2 pi i k.r_j) S_Z(k)) k
  alpha reading: alpha = sqrt(pi k_c / r_c), k_c = min N_mu/(2 L_mu),
  r_c = min L_mu / 2 (balances the real- and reciprocal-space truncations so the
  minimum image suffices, as Sec. 2.6.3 asks).
Electron-ion (Sec. 2.6.5):
    E^ie = int n V^ie + E_alpha,
    E_alpha = <n> sum_s N_s lim_{k->0}[V^_s(k) + Z_s/(pi k^2)] = <n> sum_s N_s 2 pi Z_s r_c^2
    F^ie_j = -(2 pi/|Omega|) sum_{k in box} V^_s(k) Im[conj(n^(k)) exp(-2 pi i k.r_j)] k
  (the exact derivative -dE^ie/dr_j of the discrete energy; the printed form
  omits 1/|Omega| and its sign depends on the potential sign convention).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from .grid import Grid

TWO_PI = 2.0 * math.pi


def structure_factors(g: Grid, pos: np.ndarray, species: np.ndarray, n_species: int):
    """Per-species S_s(k) on the full box, shape (n_species, Nx, Ny, Nz).
    Direct sum over atoms of the plane-wave phase."""
    S = np.zeros((n_species,) + g.shape, dtype=np.complex128)
    for j in range(pos.shape[0]):
        kr = g.k[0] * pos[j, 0] + g.k[1] * pos[j, 1] + g.k[2] * pos[j, 2]
        S[species[j]] += np.exp(-1j * TWO_PI * kr)
    return S


class Tabulated:
    """A species' tabulated non-Coulomb form factor D(q_i), q_i = i dq (1/bohr)."""

    def __init__(self, table, dq):
        self.table = np.asarray(table, dtype=np.float64).reshape(-1)
        self.dq = float(dq)

    def interpolate(self, q):
        """(D(q), dD/dq) by the local cubic through nodes i-1..i+2, i = floor(q/dq)."""
        x = np.asarray(q, dtype=np.float64) / self.dq
        i = np.floor(x).astype(np.int64)
        t = x - i
        f = self.table
        if np.any(i + 2 >= f.size):
            raise ValueError("form factor table too short for this grid")
        nodes = [np.where(i == 0, 1, i - 1), i, i + 1, i + 2]  # node -1 mirrors node 1
        offs = [-1.0, 0.0, 1.0, 2.0]
        val = np.zeros_like(t)
        der = np.zeros_like(t)
        for a in range(4):
            # Lagrange basis polynomial of node a on the offsets -1, 0, 1, 2
            num = np.ones_like(t)
            den = 1.0
            dnum = np.zeros_like(t)
            for b in range(4):
                if b == a:
                    continue
                # product rule for the derivative of prod_b (t - o_b)
                dnum = dnum * (t - offs[b]) + num
                num = num * (t - offs[b])
                den *= offs[a] - offs[b]
            val += f[nodes[a]] * num / den
            der += f[nodes[a]] * dnum / den
        return val, der / self.dq


def form_factor(g: Grid, Z: float, rc) -> np.ndarray:
    """V^_s(|k|) on the box, zero at k = 0; rc is the empty-core radius or a Tabulated."""
    V = np.zeros(g.shape)
    q = g.kabs[g.nonzero]
    if isinstance(rc, Tabulated):
        V[g.nonzero] = rc.interpolate(q)[0] - Z / (math.pi * q * q)
    else:
        V[g.nonzero] = -Z * np.cos(TWO_PI * q * rc) / (math.pi * q * q)
    return V


def form_factor_dq(g: Grid, Z: float, rc) -> np.ndarray:
    """dV^_s/d|k| (zero at k = 0, where it is not used)."""
    D = np.zeros(g.shape)
    q = g.kabs[g.nonzero]
    if isinstance(rc, Tabulated):
        D[g.nonzero] = rc.interpolate(q)[1] + 2.0 * Z / (math.pi * q ** 3)
        return D
    a = TWO_PI * q * rc
    D[g.nonzero] = Z * (TWO_PI * rc * np.sin(a) / (q * q) + 2.0 * np.cos(a) / q ** 3) / math.pi
    return D


def form_factor_k0(Z: float, rc) -> float:
    """lim_{k->0} [V^_s(k) + Z/(pi k^2)]: 2 pi Z r_c^2 for the empty core, D(0) for a table."""
    if isinstance(rc, Tabulated):
        return float(rc.table[0])
    return TWO_PI * Z * rc ** 2


def ionic_potential_hat(g: Grid, S: np.ndarray, Z, rc) -> np.ndarray:
    V = np.zeros(g.shape, dtype=np.complex128)
    for s in range(S.shape[0]):
        V += form_factor(g, Z[s], rc[s]) * S[s]
    return V


def ionic_potential(g: Grid, S, Z, rc) -> np.ndarray:
    return g.inverse(ionic_potential_hat(g, S, Z, rc))


def charge_structure_factor(S, Z) -> np.ndarray:
    return sum(Z[s] * S[s] for s in range(S.shape[0]))


# ---------------- Ewald ----------------
def ewald_alpha(g: Grid) -> float:
    kc = min(n / (2.0 * L) for n, L in zip(g.shape, g.cell))
    rc = min(L / 2.0 for L in g.cell)
    return math.sqrt(math.pi * kc / rc)


def min_image(d: np.ndarray, cell) -> np.ndarray:
    L = np.asarray(cell)
    return d - L * np.round(d / L)


def ewald(g: Grid, pos, Zj, SZ, alpha=None, atoms=None):
    """Return dict with U_pp, U_pm, U_je, U_ii and forces F_pp, F_pm (N_i x 3).
    With `atoms` given, F_pm is formed only for those atoms (rows of the others
    stay zero): the reciprocal-space sum per atom is the costly part."""
    if alpha is None:
        alpha = ewald_alpha(g)
    n = pos.shape[0]
    U_pp = 0.0
    F_pp = np.zeros((n, 3))
    for j in range(n):
        d = min_image(pos[j] - pos, g.cell)  # r_j - r_l
        r = np.sqrt(np.sum(d * d, axis=1))
        mask = np.arange(n) != j
        rr = r[mask]
        zz = Zj[j] * Zj[mask]
        U_pp += 0.5 * float(np.sum(zz * erfc(alpha * rr) / rr))
        coef = zz * (erfc(alpha * rr) / rr + 2.0 * alpha / math.sqrt(math.pi) * np.exp(-(alpha * rr) ** 2)) / rr ** 2
        F_pp[j] = np.sum(coef[:, None] * d[mask], axis=0)
    Va = np.zeros(g.shape)
    k2 = g.k2[g.nonzero]
    Va[g.nonzero] = np.exp(-(math.pi ** 2) * k2 / alpha ** 2) / (math.pi * k2)
    U_pm = 0.5 / g.volume * float(np.sum(Va * np.abs(SZ) ** 2)) - alpha / math.sqrt(math.pi) * float(np.sum(Zj ** 2))
    Q = float(np.sum(Zj))
    U_je = -math.pi * Q * Q / (2.0 * alpha ** 2 * g.volume)
    F_pm = np.zeros((n, 3))
    for j in (range(n) if atoms is None else atoms):
        kr = g.k[0] * pos[j, 0] + g.k[1] * pos[j, 1] + g.k[2] * pos[j, 2]
        im = np.imag(np.exp(1j * TWO_PI * kr) * SZ) * Va
        for a in range(3):
            F_pm[j, a] = Zj[j] * TWO_PI / g.volume * float(np.sum(im * g.k[a]))
    return dict(alpha=alpha, U_pp=U_pp, U_pm=U_pm, U_je=U_je, U_ii=U_pp + U_pm + U_je,
                F_pp=F_pp, F_pm=F_pm)


def ewald_stress_trace_printed(g: Grid, pos, Zj, SZ, alpha):
    """-1/3 tr(sigma^pp + sigma^pm + sigma^je) with the tensors exactly as
    printed in Sec. 2.6.3 (alpha held fixed).  Cross-check of P_ii only."""
    n = pos.shape[0]
    tr_pp = 0.0
    for j in range(n):
        d = min_image(pos[j] - pos[j + 1:], g.cell)
        r = np.sqrt(np.sum(d * d, axis=1))
        coef = Zj[j] * Zj[j + 1:] * (erfc(alpha * r) / r + 2.0 * alpha / math.sqrt(math.pi) * np.exp(-(alpha * r) ** 2))
        tr_pp += float(np.sum(coef * 1.0))  # r_mu r_mu / r^2 summed over mu = 1
    tr_pp *= -1.0 / g.volume
    k2 = g.k2[g.nonzero]
    Va = np.exp(-(math.pi ** 2) * k2 / alpha ** 2) / (math.pi * k2)
    S2 = np.abs(SZ[g.nonzero]) ** 2
    tr_pm = 0.5 / g.volume ** 2 * float(np.sum(Va * S2 * (2.0 * k2 * (math.pi ** 2 / alpha ** 2 + 1.0 / k2) - 3.0)))
    Q = float(np.sum(Zj))
    tr_je = 3.0 * math.pi * Q * Q / (2.0 * alpha ** 2 * g.volume ** 2)
    return -(tr_pp + tr_pm + tr_je) / 3.0


# ---------------- electron-ion ----------------
def e_alpha(g: Grid, species, Z, rc) -> float:
    Ne = float(sum(Z[s] for s in species))
    nbar = Ne / g.volume
    return nbar * float(sum(form_factor_k0(Z[s], rc[s]) for s in species))


def electron_ion_energy(g: Grid, n, Vie, species, Z, rc) -> float:
    return g.integrate(n * Vie) + e_alpha(g, species, Z, rc)


def electron_ion_forces(g: Grid, nhat, pos, species, Z, rc, atoms=None):
    """F^ie_j for j in `atoms` (default all)."""
    if atoms is None:
        atoms = range(pos.shape[0])
    atoms = list(atoms)
    Vs = [form_factor(g, Z[s], rc[s]) for s in range(len(Z))]
    F = np.zeros((len(atoms), 3))
    cn = np.conj(nhat)
    for i, j in enumerate(atoms):
        kr = g.k[0] * pos[j, 0] + g.k[1] * pos[j, 1] + g.k[2] * pos[j, 2]
        t = Vs[species[j]] * np.imag(cn * np.exp(-1j * TWO_PI * kr))
        for a in range(3):
            F[i, a] = -TWO_PI / g.volume * float(np.sum(t * g.k[a]))
    return F


def electron_ion_pressure(g: Grid, nhat, S, Eie, Z, rc) -> float:
    """P_ie = E^ie/|Omega| + 1/(3|Omega|^2) Re sum_k conj(n^) |k| V^_s'(|k|) S_s(k)."""
    acc = 0.0
    for s in range(S.shape[0]):
        acc += float(np.real(np.sum(np.conj(nhat) * g.kabs * form_factor_dq(g, Z[s], rc[s]) * S[s])))
    return Eie / g.volume + acc / (3.0 * g.volume ** 2)
