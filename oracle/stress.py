"""Oracle (test infrastructure only): the stress tensor of Sec. 2.6,
Sigma = sigma^i + sigma^e + sigma^ii + sigma^ee + sigma^ie, with P = -tr(Sigma)/3.

Each term is sigma_{mu nu} = (1/|Omega|) dE/d eps_{mu nu}: the derivative of the
corresponding discrete energy under a homogeneous strain of the cell at fixed
fractional ion coordinates and fixed grid counts (so k . r is unchanged,
k -> (1 + eps)^{-T} k, |Omega| -> det(1 + eps) |Omega|, and the density scales
as 1/det so that the electron count stays N_e).  At the converged density the
free energy is stationary under number-conserving changes of n, so the total
is dF/d eps.  Terms (box sums are over the full box, k != 0 where the kernel
is singular; conj(.) is complex conjugation):

  sigma^i   = -(1/|Omega|) sum_j m_j v_mu v_nu                      (Sec. 2.6.1)
  sigma^TF  = -(1/|Omega|) int p0 delta_{mu nu}  (f0 - n df0/dn = -p0) (Sec. 2.6.2)
  sigma^vW  = -(lambda (2 pi)^2/|Omega|^2) sum_k k_mu k_nu |s^(k)|^2,
              s = sqrt(n): F_vW = (lambda/2)(1/|Omega|) sum (2 pi k)^2 |s^|^2
              with s^ -> sqrt(det) s^ and k^2 -> k^2 - 2 eps_{mu nu} k_mu k_nu
  sigma^xc  = -(1/|Omega|) int n (v_xc - eps_xc) delta_{mu nu}  (local)
  sigma^ee  = (1/(2|Omega|^2)) sum_{k!=0} |n^|^2/(pi k^2) [2 k_mu k_nu/k^2 - delta] (Sec. 2.6.4)
  sigma^ie  = -(E^ie/|Omega|) delta
              - (1/|Omega|^2) Re sum_{k!=0} conj(n^) (k_mu k_nu/|k|) sum_s V_s'(|k|) S_s   (Sec. 2.6.5)
  sigma^pp  = -(1/|Omega|) sum_{j<l} Z_j Z_l [erfc(a d)/d + 2a/sqrt(pi) e^{-a^2 d^2}] d_mu d_nu/d^2
  sigma^pm  = (1/(2|Omega|^2)) sum_{k!=0} V_a |S_Z|^2 [2 k_mu k_nu (pi^2/a^2 + 1/k^2) - delta]
  sigma^je  = (pi Q^2/(2 a^2 |Omega|^2)) delta                      (Sec. 2.6.3, alpha held fixed)

The vW and xc tensors are not printed in the paper (it points to the
literature); they follow from the same strain derivative of their energies.
With the Ewald parameter held fixed the ion-ion tensor's trace equals
U^ii/(3|Omega|) only up to the Ewald truncation (U^ii does not depend on alpha
beyond it).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from . import fd
from . import functional as fn
from . import ionic

TERMS = ("i", "TF", "vW", "xc", "ee", "ie", "ii")


def _kk(g):
    """k_mu k_nu on the full box, shape (3, 3) + grid."""
    k = g.k
    return np.array([[k[a] * k[b] for b in range(3)] for a in range(3)])


def stress(sys, ion, res, vel=None, alpha=None, E_ie=None):
    """Dict term -> 3x3 tensor (Hartree/bohr^3) at the converged SCFResult `res`."""
    g = sys.grid
    V = g.volume
    I3 = np.eye(3)
    n = res.n
    nhat = g.forward(n)
    kk = _kk(g)
    nz = g.nonzero
    out = {}
    # ions' kinetic term
    if vel is None:
        out["i"] = np.zeros((3, 3))
    else:
        m = np.array([sys.mass[s] for s in sys.species])
        v = np.asarray(vel, dtype=np.float64).reshape(-1, 3)
        out["i"] = -np.einsum("j,ja,jb->ab", m, v, v) / V
    # Thomas-Fermi
    p0 = fd.pressure0(res.eta, sys.kT)
    out["TF"] = -g.integrate(p0) / V * I3
    # von Weizsaecker
    if sys.lam != 0.0:
        shat = g.forward(np.sqrt(n))
        w = np.abs(shat) ** 2
        out["vW"] = -sys.lam * (2.0 * math.pi) ** 2 / V ** 2 * np.array(
            [[float(np.sum(kk[a, b] * w)) for b in range(3)] for a in range(3)])
    else:
        out["vW"] = np.zeros((3, 3))
    # exchange-correlation (local)
    if sys.xc:
        exc, vxc = fn.xc_terms(n)
        out["xc"] = -g.integrate(n * (vxc - exc)) / V * I3
    else:
        out["xc"] = np.zeros((3, 3))
    # Hartree
    h = np.zeros(g.shape)
    h[nz] = np.abs(nhat[nz]) ** 2 / (math.pi * g.k2[nz])
    k2s = np.where(nz, g.k2, 1.0)
    out["ee"] = np.array([[float(np.sum(h * (2.0 * kk[a, b] / k2s - (1.0 if a == b else 0.0))))
                           for b in range(3)] for a in range(3)]) / (2.0 * V ** 2)
    # electron-ion
    if E_ie is None:
        E_ie = ionic.electron_ion_energy(g, n, ion.Vie, sys.species, sys.Z, sys.rc)
    acc = np.zeros(g.shape)
    for s in range(ion.S.shape[0]):
        acc += np.real(np.conj(nhat) * ion.S[s]) * ionic.form_factor_dq(g, sys.Z[s], sys.rc[s])
    kabs = np.where(nz, g.kabs, 1.0)
    acc = np.where(nz, acc / kabs, 0.0)
    out["ie"] = -E_ie / V * I3 - np.array([[float(np.sum(acc * kk[a, b])) for b in range(3)]
                                          for a in range(3)]) / V ** 2
    # ion-ion (Ewald, alpha fixed)
    out["ii"] = ewald_stress(g, sys.pos, sys.Zj, ion.SZ, alpha if alpha is not None else
                             (sys.ewald_alpha if sys.ewald_alpha > 0 else ionic.ewald_alpha(g)))
    return out


def ewald_stress(g, pos, Zj, SZ, alpha):
    """sigma^pp + sigma^pm + sigma^je as printed in Sec. 2.6.3 (alpha fixed)."""
    V = g.volume
    n = pos.shape[0]
    pp = np.zeros((3, 3))
    for j in range(n):
        d = ionic.min_image(pos[j] - pos[j + 1:], g.cell)
        r = np.sqrt(np.sum(d * d, axis=1))
        coef = Zj[j] * Zj[j + 1:] * (erfc(alpha * r) / r + 2.0 * alpha / math.sqrt(math.pi)
                                     * np.exp(-(alpha * r) ** 2)) / r ** 2
        pp -= np.einsum("l,la,lb->ab", coef, d, d)
    pp /= V
    nz = g.nonzero
    k2 = np.where(nz, g.k2, 1.0)
    Va = np.where(nz, np.exp(-(math.pi ** 2) * k2 / alpha ** 2) / (math.pi * k2), 0.0)
    w = Va * np.abs(SZ) ** 2
    kk = _kk(g)
    pm = np.array([[float(np.sum(w * (2.0 * kk[a, b] * (math.pi ** 2 / alpha ** 2 + 1.0 / k2)
                                      - (1.0 if a == b else 0.0))))
                    for b in range(3)] for a in range(3)]) / (2.0 * V ** 2)
    Q = float(np.sum(Zj))
    je = math.pi * Q * Q / (2.0 * alpha ** 2 * V ** 2) * np.eye(3)
    return pp + pm + je


def total(terms):
    return sum(terms[t] for t in TERMS)
