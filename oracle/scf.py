"""Oracle (test infrastructure only): the SCF density iteration, Sec. 2.5.

One iteration, with input density n_i (Sec. 2.5 and its subsections):
  1. V_i = V^ie + V_H[n_i] + v_xc(n_i) + v_vW[n_i]   (vW and xc lagged like
     Hartree: they enter the effective potential evaluated at n_i)
  2. mu solves N(mu) = int c_n I_{1/2}((mu - V_i)/kT) = N_e (eq. newtonmu), by
     Newton's method safeguarded with bisection inside a bracket that holds
     the root (N is strictly increasing in mu, so the root is unique)
  3. n_a = c_n I_{1/2}((mu - V_i)/kT),  Delta n = n_i - n_a
  4. stop when ||Delta n||_2 / ||n_a||_2 < tol (relative discrete L2 norm);
     the result is n_a at that mu
  5. mixing weight (Sec. 2.5.2): n_o = n_a + w Delta n.  Fixed mixing uses
     w = w_fixed throughout.  More mixing uses w_fixed until it is switched
     on, then w = U / (U + K) clamped to [0, 0.995], with
        U = -int (dF/dn at n_a) Delta n = int (V_i - V_eff[n_a]) Delta n
        K = int kT (eta(n_i) - eta_a) Delta n,  eta(n) = I_{1/2}^{-1}(n / c_n)
     Readings (the paper states U only for the Hartree term and says adding
     the other potential terms is straightforward; its K is the second-order
     form int Delta n^2 / (dn_a/dmu); it switches More's weight on "after a
     few iterations, once the chemical potential fluctuations are small"):
     U keeps every potential term -- Hartree, xc and vW -- as the secant
     difference above (with vW present the Hartree-only U drives the stiff
     short-wavelength vW modes unstable); K is taken as the same kind of secant
     of the Thomas-Fermi potential kT eta(n), which equals the paper's K to
     second order in Delta n but stays bounded where n_i / n_a is large (low
     density regions at low T, where the second-order K grows like n_i / n_a,
     drives w to 0 and the iteration diverges); the switch happens at the first
     iteration t >= warmup at which either the second-order expansion behind
     the weight holds pointwise, max_r |Delta n| / n_a <= more_trust (0.5), or
     mu moved by at most MU_SETTLED kT since the previous iteration, and is
     never undone; and the weight may fall by at most W_MAX_DROP (0.05) per
     iteration (where xc makes U small or negative in low-density regions the
     quadratic model sends w to 0 in one step and the iteration diverges).
     mixing="more_printed" takes the weight exactly as printed instead: U the
     Hartree term alone, U = int int dn dn' / |r - r'|, and the second-order
     K = int dn^2 / (dn_a/dmu), w = U / (U + K) clamped to [0, 0.995], with the
     same switch and no bound on its fall.
  6. n_o = n_a + w Delta n becomes the next n_i.

Initial densities (Sec. 2.5 and 2.5.1):
  uniform     n_0 = N_e / |Omega|
  one-center  g^ = n^ / S_Z taken as a least-squares fit per |k|^2 shell
              (g^(shell) = sum Re(n^ conj S_Z) / sum |S_Z|^2 over the shell),
              n^_i = g^ S_Z(new positions), floored at GUESS_FLOOR n_0 and
              rescaled to N_e; falls back to uniform if the floor added more
              than MAX_FLOOR_CHARGE of the charge.  (The superposition rings
              slightly negative between the ions; a floor near zero would make
              sqrt(n), and with it the von Weizsaecker potential of the guess,
              nearly singular there.)  Shells whose sum |S_Z|^2 is below SHELL_CUT x
              (shell size) x sum_j Z_j^2 get g^ = 0: near a perfect lattice
              S_Z is tiny off the lattice's own shells, and n^ / S_Z there is
              the nonlinear response, not a one-center profile (random
              positions give sum |S_Z|^2 ~ (shell size) x sum Z_j^2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import fd
from . import functional as fn
from . import ionic
from .grid import Grid

GUESS_FLOOR = 1e-3  # floor of the one-center guess, in units of n_0
MAX_FLOOR_CHARGE = 1e-6  # uniform instead when the floor adds more than this fraction of N_e
SHELL_CUT = 1e-12  # shells with less structure-factor weight get no one-center profile
# More's weight may fall by at most this much from one iteration to the next
W_MAX_DROP = 0.05


@dataclass
class System:
    cell: tuple
    shape: tuple
    pos: np.ndarray  # (N_i, 3) bohr
    species: np.ndarray  # (N_i,) int
    Z: tuple  # per species
    rc: tuple  # per species, bohr
    mass: tuple  # per species, electron masses
    kT: float  # Hartree
    lam: float = 0.2  # von Weizsaecker coefficient
    xc: bool = True  # Dirac + PZ81 LDA
    ewald_alpha: float = 0.0  # Ewald splitting; <= 0: the automatic choice

    def __post_init__(self):
        self.pos = np.asarray(self.pos, dtype=np.float64).reshape(-1, 3)
        self.species = np.asarray(self.species, dtype=np.int64).reshape(-1)
        self.Z = tuple(float(z) for z in self.Z)
        # per species: empty-core radius, or a tabulated form factor (ionic.Tabulated)
        self.rc = tuple(r if isinstance(r, ionic.Tabulated) else float(r) for r in self.rc)
        self.mass = tuple(float(m) for m in self.mass)
        self.grid = Grid(self.cell, self.shape)
        self.Zj = np.array([self.Z[s] for s in self.species])
        self.Ne = float(np.sum(self.Zj))

    def with_positions(self, pos):
        return System(self.cell, self.shape, pos, self.species, self.Z, self.rc, self.mass,
                      self.kT, self.lam, self.xc, self.ewald_alpha)


@dataclass
class Ionic:
    S: np.ndarray  # per-species structure factor, full box
    SZ: np.ndarray
    Vie: np.ndarray  # real space


def ionic_setup(sys: System) -> Ionic:
    g = sys.grid
    S = ionic.structure_factors(g, sys.pos, sys.species, len(sys.Z))
    SZ = ionic.charge_structure_factor(S, sys.Z)
    Vie = ionic.ionic_potential(g, S, sys.Z, sys.rc)
    return Ionic(S, SZ, Vie)


def effective_potential(sys: System, ion: Ionic, n: np.ndarray):
    """V_i = V^ie + V_H[n] + v_xc(n) + v_vW[n]; returns (V, nhat)."""
    g = sys.grid
    nhat = g.forward(n)
    V = ion.Vie + fn.hartree_potential(g, nhat)
    if sys.xc:
        V = V + fn.xc_terms(n)[1]
    if sys.lam != 0.0:
        V = V + fn.vw_terms(g, n, sys.lam)[0]
    return V, nhat


def electron_count(sys: System, V, mu):
    eta = (mu - V) / sys.kT
    v = fd.fd_integrals(eta, ("m12", "p12"))
    cn = fd.c_n(sys.kT)
    N = sys.grid.dv * cn * float(np.sum(v["p12"]))
    dN = sys.grid.dv * cn / (2.0 * sys.kT) * float(np.sum(v["m12"]))
    return N, dN


_ETA0_CACHE = {}


def uniform_eta(sys: System) -> float:
    """eta_0 = I_{1/2}^{-1}(n_0 / c_n) of the uniform gas at this density and temperature."""
    key = (sys.Ne, sys.grid.volume, sys.kT)
    if key not in _ETA0_CACHE:
        _ETA0_CACHE[key] = fd.I_p12_inverse(sys.Ne / sys.grid.volume / fd.c_n(sys.kT))
    return _ETA0_CACHE[key]


def solve_mu(sys: System, V, mu0=None, rtol=1e-14, max_iter=200):
    """Chemical potential with int n = N_e (eq. newtonmu).  Returns (mu, newton_iters)."""
    kT, Ne = sys.kT, sys.Ne
    x0 = uniform_eta(sys)
    lo = float(np.min(V)) + kT * x0
    hi = float(np.max(V)) + kT * x0
    if mu0 is None or not (lo <= mu0 <= hi):
        mu0 = float(np.mean(V)) + kT * x0
    mu = mu0
    for it in range(1, max_iter + 1):
        N, dN = electron_count(sys, V, mu)
        f = N - Ne
        if abs(f) <= rtol * Ne:
            return mu, it
        if f > 0:
            hi = mu
        else:
            lo = mu
        mn = mu - f / dN
        if not (lo < mn < hi):
            mn = 0.5 * (lo + hi)
        if abs(mn - mu) <= 1e-15 * (abs(mu) + kT):
            return mn, it
        mu = mn
    raise RuntimeError("mu search did not converge")


def shell_keys(g: Grid) -> np.ndarray:
    mx, my, mz = g.m
    cubic = len(set(g.cell)) == 1 and len(set(g.shape)) == 1
    if cubic:
        return (mx * mx + my * my + mz * mz).astype(np.int64)
    P = max(g.shape) ** 2 // 4 + 1
    return ((mx * mx).astype(np.int64) * P + my * my) * P + mz * mz


def one_center_profile(sys: System, nhat_prev: np.ndarray, SZ_prev: np.ndarray):
    """g^ per shell from the previous converged spectrum; returns (keys, ghat per point)."""
    g = sys.grid
    keys = shell_keys(g).reshape(-1)
    num = np.real(nhat_prev * np.conj(SZ_prev)).reshape(-1)
    den = (np.abs(SZ_prev) ** 2).reshape(-1)
    uk, inv = np.unique(keys, return_inverse=True)
    snum = np.bincount(inv, weights=num, minlength=uk.size)
    sden = np.bincount(inv, weights=den, minlength=uk.size)
    cnt = np.bincount(inv, minlength=uk.size)
    thresh = SHELL_CUT * cnt * float(np.sum(sys.Zj ** 2))
    gsh = np.where(sden > thresh, snum / np.where(sden > 0, sden, 1.0), 0.0)
    return gsh[inv].reshape(g.shape)


def initial_density(sys: System, ion: Ionic, kind="uniform", prev=None):
    """Returns (n_i, used_fallback)."""
    g = sys.grid
    n0 = sys.Ne / g.volume
    if kind == "uniform" or prev is None:
        return np.full(g.shape, n0), kind != "uniform"
    if kind == "one_center":
        nhat_prev, SZ_prev = prev
        ghat = one_center_profile(sys, nhat_prev, SZ_prev)
        n = g.inverse(ghat * ion.SZ)
        raw = g.integrate(n)
        n = np.maximum(n, GUESS_FLOOR * n0)
        added = g.integrate(n) - raw
        if abs(added) > MAX_FLOOR_CHARGE * sys.Ne:
            return np.full(g.shape, n0), True
        n = n * (sys.Ne / g.integrate(n))
        return n, False
    if kind == "given":
        return np.asarray(prev, dtype=np.float64).copy(), False
    raise ValueError(kind)


@dataclass
class SCFResult:
    n: np.ndarray  # converged active density n_a
    eta: np.ndarray  # (mu - V_i)/kT at convergence
    mu: float
    V: np.ndarray  # V_i of the last iteration
    iters: int
    residual: float
    converged: bool
    history: list = field(default_factory=list)
    newton: list = field(default_factory=list)
    weights: list = field(default_factory=list)
    used_fallback: bool = False


# More's weight may switch on once mu moves by at most this fraction of kT
# between iterations (the paper's "mu fluctuations are small")
MU_SETTLED = 0.02


def scf(sys: System, ion: Ionic, n_init: np.ndarray, mixing="more", tol=1e-10, max_iter=5000,
        warmup=3, w_fixed=0.95, more_trust=0.5, mu0=None) -> SCFResult:
    g = sys.grid
    n_i = n_init.copy()
    mu = mu0
    hist, newt, ws = [], [], []
    cn = fd.c_n(sys.kT)
    more_on = False
    r = float("inf")
    n_a = eta = V = None
    for t in range(max_iter):
        V, _ = effective_potential(sys, ion, n_i)
        mu_prev = mu
        mu, nit = solve_mu(sys, V, mu)
        newt.append(nit)
        eta = (mu - V) / sys.kT
        v = fd.fd_integrals(eta, ("m12", "p12"))
        n_a = cn * v["p12"]
        dn = n_i - n_a
        r = math.sqrt(float(np.sum(dn * dn)) / float(np.sum(n_a * n_a)))
        hist.append(r)
        if r < tol:
            return SCFResult(n_a, eta, mu, V, t + 1, r, True, hist, newt, ws)
        if mixing in ("more", "more_printed") and not more_on and t >= warmup:
            more_on = (float(np.max(np.abs(dn) / n_a)) <= more_trust
                       or (mu_prev is not None and abs(mu - mu_prev) <= MU_SETTLED * sys.kT))
        if more_on and mixing == "more_printed":
            # the weight exactly as printed (Sec. 2.5.2): U the Hartree interaction of
            # dn with itself, K = int dn^2 / (dn_a/dmu), w = U / (U + K) in [0, 0.995]
            U = 2.0 * fn.hartree_energy(g, g.forward(dn))
            chi = cn / (2.0 * sys.kT) * v["m12"]
            K = g.integrate(dn * dn / chi)
            w = min(max(U / (U + K), 0.0), 0.995)
        elif more_on:
            # U and K are the secants of the interaction and of the Thomas-Fermi
            # potential between n_a and n_i along dn (K -> int dn^2/chi as dn -> 0)
            Va, _ = effective_potential(sys, ion, n_a)
            U = g.integrate((V - Va) * dn)
            eta_i = fd.I_p12_inverse_array(n_i / cn, eta)
            K = g.integrate(sys.kT * (eta_i - eta) * dn)
            w = min(max(U / (U + K), 0.0), 0.995)
            if ws:
                w = max(w, ws[-1] - W_MAX_DROP)
        else:
            w = w_fixed
        ws.append(w)
        n_i = n_a + w * dn
    return SCFResult(n_a, eta, mu, V, max_iter, r, False, hist, newt, ws)


def scf_anderson(sys: System, ion: Ionic, n_init: np.ndarray, tol=1e-12, max_iter=2000, history=8, beta=0.5,
                 mu0=None) -> SCFResult:
    """The same fixed point (the Euler equation's solution, n_i = n_a) reached by
    Anderson's acceleration of the map n_i -> n_a (Anderson 1965, in the
    least-squares form of Pulay's DIIS): a robust generic iteration used only to
    produce reference values of large cells quickly; the paper's own iteration is
    `scf` above.  Residual f = n_a - n_i; with the last `history` differences of
    inputs (dX) and residuals (dF), gamma = argmin ||f - dF gamma||_2 and
    n_next = n_i + beta f - (dX + beta dF) gamma.  A step that would leave a
    non-positive density is replaced by plain mixing n_i + beta f (a convex
    combination of two positive densities) and the history restarts.  The stop
    test and the result are those of `scf`: ||n_i - n_a||_2/||n_a||_2 < tol,
    result n_a at its mu."""
    cn = fd.c_n(sys.kT)
    x = n_init.copy()
    mu = mu0
    hist, newt = [], []
    dX, dF = [], []
    x_prev = f_prev = None
    r = float("inf")
    n_a = eta = V = None
    for t in range(max_iter):
        V, _ = effective_potential(sys, ion, x)
        mu, nit = solve_mu(sys, V, mu)
        newt.append(nit)
        eta = (mu - V) / sys.kT
        n_a = cn * fd.fd_integrals(eta, ("p12",))["p12"]
        f = n_a - x
        r = math.sqrt(float(np.sum(f * f)) / float(np.sum(n_a * n_a)))
        hist.append(r)
        if r < tol:
            return SCFResult(n_a, eta, mu, V, t + 1, r, True, hist, newt, [])
        if x_prev is not None:
            dX.append((x - x_prev).reshape(-1))
            dF.append((f - f_prev).reshape(-1))
            if len(dX) > history:
                dX.pop(0)
                dF.pop(0)
        x_prev, f_prev = x, f
        step = x + beta * f
        if dX:
            A = np.stack(dF, axis=1)
            gamma = np.linalg.lstsq(A, f.reshape(-1), rcond=None)[0]
            B = np.stack(dX, axis=1) + beta * A
            cand = step - (B @ gamma).reshape(x.shape)
            if float(np.min(cand)) > 0.0:
                step = cand
            else:
                dX, dF = [], []
        x = step
    return SCFResult(n_a, eta, mu, V, max_iter, r, False, hist, newt, [])
