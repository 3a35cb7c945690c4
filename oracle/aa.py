"""Oracle (test infrastructure only): the average-atom pseudopotential of
Sec. 2.4 and the energy correction Delta E_AA.

Average atom: one nucleus of charge Z at the centre of the Wigner-Seitz
sphere, 4/3 pi r_ws^3 = 1/rho (rho the ionic number density), filled with a
finite-temperature Thomas-Fermi electron density (+ the same LDA xc as the
grid path when xc is on), neutral inside the sphere:
    n(r) = c_n I_{1/2}((mu - V(r))/kT),   int_0^{r_ws} 4 pi r^2 n = Z,
    V(r) = -Z/r + V_H(r) + v_xc(n(r)),
    V_H(r) = (1/r) int_0^r 4 pi x^2 n dx + int_r^{r_ws} 4 pi x n dx
(V is the electron's potential energy, the sign convention of the grid path).
Solved on a radial grid uniform in u = ln r from r_min to r_ws, integrals by
the trapezoid rule in u (int f dr = int f r du), by damped fixed-point
iteration of V_H + v_xc with mu fixed by the neutrality at each step.

Pseudo-density (the paper's three constraints): inside r_cut
    n~(r) = exp(a + b r^2 + c r^4),
with n~(r_cut) = n(r_cut), n~'(r_cut) = n'(r_cut) and the same charge inside
r_cut; n~ = n outside.  The first two fix a and b linearly in c; the charge
fixes c (one monotone equation, bracketed root).  n' is the derivative of the
TF relation, n' = (dn/deta) eta', eta' = -(Z/r^2 - Q(r)/r^2 + v_xc'(n) n')/kT
solved for n' (Q(r) the electron charge inside r).

Pseudopotential (Sec. 2.4): inside r_cut the potential whose TF + Hartree + xc
response is n~,
    V~(r) = mu - kT I_{1/2}^{-1}(n~/c_n) - v_xc(n~) - V_H[n~](r),
and the nuclear Coulomb potential -Z/r outside (continuous at r_cut by norm
conservation).  Its non-Coulomb part dV = V~ + Z/r vanishes outside r_cut, so
its Fourier transform (ordinary frequency q = |k|) is
    D(q) = 4 pi int_0^{r_cut} dV(r) r^2 sin(2 pi q r)/(2 pi q r) dr,
the tabulated form factor of the grid path (V^(q) = -Z/(pi q^2) + D(q)), and
D(0) = 4 pi int dV r^2 dr the k = 0 term of E^ie.

Delta E_AA = E[n; -Z/r] - E[n~; V~] per atom, the internal energies of the
two average atoms: K_e + int n V_ion + (1/2) int n V_H + int n eps_xc, with
K_e = (3/2) int p0 (Sec. 2.6.2); it is added to the grid path's internal
energy per atom.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import fd
from . import functional as fn


@dataclass
class RadialGrid:
    r: np.ndarray
    w: np.ndarray  # trapezoid weights in u = ln r, times r: int f dr = sum w f

    @staticmethod
    def make(r_ws, n=2001, r_min_frac=1e-7):
        u = np.linspace(math.log(r_min_frac * r_ws), math.log(r_ws), n)
        r = np.exp(u)
        du = u[1] - u[0]
        w = np.full(n, du) * r
        w[0] *= 0.5
        w[-1] *= 0.5
        return RadialGrid(r, w)

    def integral(self, f):
        return float(np.sum(self.w * f))

    def cumulative(self, f):
        """int_{r_0}^{r_i} f dr for every i (trapezoid in u)."""
        g = f * self.r
        du = math.log(self.r[1] / self.r[0])
        c = np.concatenate(([0.0], np.cumsum(0.5 * du * (g[1:] + g[:-1]))))
        return c


def hartree(grid, n):
    """V_H(r) of a spherical charge inside the sphere, and the charge Q(r) inside r."""
    r = grid.r
    Q = grid.cumulative(4.0 * math.pi * r * r * n)
    outer = grid.cumulative(4.0 * math.pi * r * n)
    return Q / r + (outer[-1] - outer), Q


def _vxc(n, xc):
    return fn.xc_terms(n)[1] if xc else np.zeros_like(n)


def _exc(n, xc):
    return fn.xc_terms(n)[0] if xc else np.zeros_like(n)


def _mu_for(grid, V, kT, Z, mu0=None):
    """mu with int 4 pi r^2 c_n I_{1/2}((mu - V)/kT) dr = Z (Newton in a bisection bracket)."""
    cn = fd.c_n(kT)
    w4 = grid.w * 4.0 * math.pi * grid.r ** 2

    def N(mu):
        v = fd.fd_integrals((mu - V) / kT, ("m12", "p12"))
        return cn * float(np.sum(w4 * v["p12"])), cn / (2.0 * kT) * float(np.sum(w4 * v["m12"]))

    lo, hi = float(np.min(V)) - 50.0 * kT, float(np.max(V)) + 1.0
    while N(lo)[0] > Z:
        lo -= 10.0 * (abs(lo) + kT)
    while N(hi)[0] < Z:
        hi += 10.0 * (abs(hi) + kT)
    mu = mu0 if (mu0 is not None and lo < mu0 < hi) else 0.5 * (lo + hi)
    for _ in range(300):
        f, df = N(mu)
        f -= Z
        if abs(f) <= 1e-14 * Z:
            return mu
        if f > 0:
            hi = mu
        else:
            lo = mu
        mn = mu - f / df if df > 0 else 0.5 * (lo + hi)
        if not (lo < mn < hi):
            mn = 0.5 * (lo + hi)
        if abs(mn - mu) <= 1e-15 * (abs(mu) + kT):
            return mn
        mu = mn
    raise RuntimeError("average-atom mu search did not converge")


@dataclass
class AverageAtom:
    grid: RadialGrid
    Z: float
    kT: float
    xc: bool
    Vion: np.ndarray  # the ionic potential the electrons feel
    n: np.ndarray
    mu: float
    VH: np.ndarray
    Q: np.ndarray
    iters: int


def solve(grid, Z, kT, Vion, xc=True, tol=1e-12, beta=0.3, max_iter=5000):
    """The self-consistent average atom in the ionic potential Vion(r)."""
    cn = fd.c_n(kT)
    r_ws = grid.r[-1]
    n = np.full(grid.r.shape, Z / (4.0 / 3.0 * math.pi * r_ws ** 3))
    VH, Q = hartree(grid, n)
    Vs = VH + _vxc(n, xc)  # the screening part of the potential
    mu = None
    for it in range(1, max_iter + 1):
        V = Vion + Vs
        mu = _mu_for(grid, V, kT, Z, mu)
        n = cn * fd.I_p12((mu - V) / kT)
        VH, Q = hartree(grid, n)
        Vs_new = VH + _vxc(n, xc)
        d = float(np.max(np.abs(Vs_new - Vs)))
        if d <= tol * max(1.0, float(np.max(np.abs(Vs_new)))):
            return AverageAtom(grid, Z, kT, xc, Vion, n, mu, VH, Q, it)
        Vs = Vs + beta * (Vs_new - Vs)
    raise RuntimeError("average atom did not converge")


def density_slope(aa):
    """n'(r) from the TF relation (see the module notes)."""
    r, n, kT = aa.grid.r, aa.n, aa.kT
    eta = fd.I_p12_inverse_array(n / fd.c_n(aa.kT))
    dndeta = fd.c_n(kT) * 0.5 * fd.I_m12(eta)
    dVion = np.gradient(aa.Vion, r) if not np.allclose(aa.Vion, -aa.Z / r) else aa.Z / r ** 2
    dVH = -aa.Q / r ** 2
    if aa.xc:
        h = 1e-6 * n
        dvxc = (fn.xc_terms(n + h)[1] - fn.xc_terms(n - h)[1]) / (2 * h)
    else:
        dvxc = np.zeros_like(n)
    # n' = dndeta * eta',  eta' = -(dVion + dVH + dvxc n')/kT
    return -dndeta * (dVion + dVH) / kT / (1.0 + dndeta * dvxc / kT)


@dataclass
class Pseudo:
    r_cut: float
    a: float
    b: float
    c: float
    n_pseudo: np.ndarray
    V_pseudo: np.ndarray
    dV: np.ndarray  # V~ + Z/r (zero outside r_cut)


def pseudo(aa, r_cut):
    """Pseudo-density and pseudopotential of the average atom (Sec. 2.4)."""
    g = aa.grid
    r = g.r
    i_c = int(np.searchsorted(r, r_cut))
    r_cut = float(r[i_c])  # the cut sits on a grid node
    slope = density_slope(aa)
    y0 = math.log(aa.n[i_c])
    y1 = slope[i_c] / aa.n[i_c]
    inside = r <= r_cut
    wq = np.where(inside, g.w, 0.0)
    wq[i_c] *= 0.5 if i_c > 0 else 1.0  # trapezoid end point at r_cut
    q_true = float(np.sum(wq * 4 * math.pi * r * r * aa.n))

    def abc(c):
        b = (y1 - 4.0 * c * r_cut ** 3) / (2.0 * r_cut)
        a = y0 - b * r_cut ** 2 - c * r_cut ** 4
        return a, b

    def charge(c):
        a, b = abc(c)
        return float(np.sum(wq * 4 * math.pi * r * r * np.exp(a + b * r * r + c * r ** 4))) - q_true

    # the exponent is y0 + (y1/(2 r_c))(r^2 - r_c^2) + c (r^2 - r_c^2)^2, so the
    # charge grows monotonically with c: bracket the root and bisect
    lo, hi = -1.0, 1.0
    while charge(lo) > 0:
        lo *= 2.0
    while charge(hi) < 0:
        hi *= 2.0
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if charge(mid) > 0:
            hi = mid
        else:
            lo = mid
        if hi - lo <= 1e-15 * max(1.0, abs(mid)):
            break
    c = 0.5 * (lo + hi)
    a, b = abc(c)
    npseudo = np.where(inside, np.exp(a + b * r * r + c * r ** 4), aa.n)
    VH, _ = hartree(g, npseudo)
    eta = fd.I_p12_inverse_array(npseudo / fd.c_n(aa.kT))
    Vp = aa.mu - aa.kT * eta - _vxc(npseudo, aa.xc) - VH
    Vp = np.where(inside, Vp, -aa.Z / r)
    dV = np.where(inside, Vp + aa.Z / r, 0.0)
    return Pseudo(r_cut, a, b, c, npseudo, Vp, dV)


def form_factor_table(aa, ps, dq, n_q):
    """D(q_i) = 4 pi int dV r^2 j0(2 pi q_i r) dr, q_i = i dq."""
    r = aa.grid.r
    out = np.empty(n_q)
    for i in range(n_q):
        x = 2.0 * math.pi * i * dq * r
        j0 = np.where(x > 0, np.sin(x) / np.where(x > 0, x, 1.0), 1.0)
        out[i] = aa.grid.integral(4.0 * math.pi * ps.dV * r * r * j0)
    return out


def energy(aa, n, Vion):
    """Internal energy of the average atom with density n in Vion."""
    g = aa.grid
    r = g.r
    w4 = 4.0 * math.pi * r * r
    eta = fd.I_p12_inverse_array(n / fd.c_n(aa.kT))
    K = 1.5 * g.integral(w4 * fd.pressure0(eta, aa.kT))
    VH, _ = hartree(g, n)
    return (K + g.integral(w4 * n * Vion) + 0.5 * g.integral(w4 * n * VH)
            + g.integral(w4 * n * _exc(n, aa.xc)))


def pseudopotential(Z, rho_ion, kT, r_cut_frac, xc=True, dq=0.01, n_q=400, n_r=2001):
    """The whole chain: average atom at ion density rho_ion (1/bohr^3) and kT,
    pseudo-density with r_cut = r_cut_frac r_ws, its form-factor table and
    Delta E_AA.  Returns (table, Delta E_AA, details)."""
    r_ws = (3.0 / (4.0 * math.pi * rho_ion)) ** (1.0 / 3.0)
    g = RadialGrid.make(r_ws, n_r)
    aa = solve(g, Z, kT, -Z / g.r, xc)
    ps = pseudo(aa, r_cut_frac * r_ws)
    table = form_factor_table(aa, ps, dq, n_q)
    dE = energy(aa, aa.n, -Z / g.r) - energy(aa, ps.n_pseudo, ps.V_pseudo)
    return table, dE, dict(aa=aa, pseudo=ps, r_ws=r_ws)
