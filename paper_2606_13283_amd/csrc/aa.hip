// The average-atom pseudopotential of Sec. 2.4 (host code): a finite-temperature
// Thomas-Fermi (+ LDA) atom in its Wigner-Seitz sphere, the smooth pseudo-density
// exp(a + b r^2 + c r^4) inside r_cut under the paper's three constraints, the
// pseudopotential whose response is that pseudo-density, its form-factor table
// for arche_params.ff_table and the energy correction Delta E_AA.
#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/arche.h"
#include "arche_internal.h"

namespace {

constexpr double PI = 3.14159265358979323846;

// radial grid uniform in u = ln r from r_min to r_ws; trapezoid in u
struct Radial {
  std::vector<double> r, w;
  double du = 0.0;
  Radial(double r_ws, int n) : r(n), w(n) {
    const double u0 = std::log(1e-7 * r_ws), u1 = std::log(r_ws);
    du = (u1 - u0) / (n - 1);
    for (int i = 0; i < n; ++i) {
      r[i] = std::exp(u0 + du * i);
      w[i] = du * r[i] * ((i == 0 || i == n - 1) ? 0.5 : 1.0);
    }
    r[n - 1] = r_ws;
    w[n - 1] = 0.5 * du * r_ws;
  }
  int size() const { return (int)r.size(); }
  double integral(const std::vector<double>& f) const {
    double s = 0.0;
    for (int i = 0; i < size(); ++i) s += w[i] * f[i];
    return s;
  }
  // int_{r_0}^{r_i} f dr
  std::vector<double> cumulative(const std::vector<double>& f) const {
    std::vector<double> c(size(), 0.0);
    for (int i = 1; i < size(); ++i) c[i] = c[i - 1] + 0.5 * du * (f[i] * r[i] + f[i - 1] * r[i - 1]);
    return c;
  }
};

// Hartree potential of a spherical charge inside the sphere, and Q(r)
void hartree(const Radial& g, const std::vector<double>& n, std::vector<double>& VH, std::vector<double>& Q) {
  const int m = g.size();
  std::vector<double> a(m), b(m);
  for (int i = 0; i < m; ++i) {
    a[i] = 4.0 * PI * g.r[i] * g.r[i] * n[i];
    b[i] = 4.0 * PI * g.r[i] * n[i];
  }
  Q = g.cumulative(a);
  const std::vector<double> outer = g.cumulative(b);
  VH.resize(m);
  for (int i = 0; i < m; ++i) VH[i] = Q[i] / g.r[i] + (outer[m - 1] - outer[i]);
}

double vxc_of(double n, bool xc) {
  if (!xc) return 0.0;
  double v;
  (void)lda_xc(n, v);
  return v;
}
double exc_of(double n, bool xc) {
  if (!xc) return 0.0;
  double v;
  return lda_xc(n, v);
}

double cn_of(double kT) { return std::pow(2.0 * kT, 1.5) / (2.0 * PI * PI); }

// mu with int 4 pi r^2 c_n I_{1/2}((mu - V)/kT) dr = Z; Newton in a bisection bracket
bool mu_for(const Radial& g, const std::vector<double>& V, double kT, double Z, double mu0, bool have_mu0,
            double* mu_out) {
  const double cn = cn_of(kT);
  auto N = [&](double mu, double* dN) {
    double s = 0.0, d = 0.0;
    for (int i = 0; i < g.size(); ++i) {
      const double x = (mu - V[i]) / kT, w4 = g.w[i] * 4.0 * PI * g.r[i] * g.r[i];
      s += w4 * host_fd(1, x);
      d += w4 * host_fd(0, x);
    }
    *dN = cn / (2.0 * kT) * d;
    return cn * s;
  };
  double vmin = V[0], vmax = V[0];
  for (double v : V) {
    vmin = std::min(vmin, v);
    vmax = std::max(vmax, v);
  }
  double lo = vmin - 50.0 * kT, hi = vmax + 1.0, dn;
  for (int k = 0; k < 200 && N(lo, &dn) > Z; ++k) lo -= 10.0 * (std::fabs(lo) + kT);
  for (int k = 0; k < 200 && N(hi, &dn) < Z; ++k) hi += 10.0 * (std::fabs(hi) + kT);
  double mu = (have_mu0 && lo < mu0 && mu0 < hi) ? mu0 : 0.5 * (lo + hi);
  for (int it = 0; it < 300; ++it) {
    double f = N(mu, &dn) - Z;
    if (std::fabs(f) <= 1e-14 * Z) {
      *mu_out = mu;
      return true;
    }
    if (f > 0)
      hi = mu;
    else
      lo = mu;
    double mn = dn > 0 ? mu - f / dn : 0.5 * (lo + hi);
    if (!(lo < mn && mn < hi)) mn = 0.5 * (lo + hi);
    if (std::fabs(mn - mu) <= 1e-15 * (std::fabs(mu) + kT)) {
      *mu_out = mn;
      return true;
    }
    mu = mn;
  }
  return false;
}

struct Atom {
  std::vector<double> n, VH, Q;
  double mu = 0.0;
  int iters = 0;
};

// self-consistent average atom in the ionic potential Vion (damped fixed point on V_H + v_xc)
bool solve_atom(const Radial& g, double Z, double kT, const std::vector<double>& Vion, bool xc, Atom& A) {
  const int m = g.size();
  const double cn = cn_of(kT), r_ws = g.r[m - 1];
  A.n.assign(m, Z / (4.0 / 3.0 * PI * r_ws * r_ws * r_ws));
  hartree(g, A.n, A.VH, A.Q);
  std::vector<double> Vs(m), V(m), Vn(m);
  for (int i = 0; i < m; ++i) Vs[i] = A.VH[i] + vxc_of(A.n[i], xc);
  bool have_mu = false;
  for (int it = 1; it <= 5000; ++it) {
    for (int i = 0; i < m; ++i) V[i] = Vion[i] + Vs[i];
    if (!mu_for(g, V, kT, Z, A.mu, have_mu, &A.mu)) return false;
    have_mu = true;
    for (int i = 0; i < m; ++i) A.n[i] = cn * host_fd(1, (A.mu - V[i]) / kT);
    hartree(g, A.n, A.VH, A.Q);
    double d = 0.0, big = 1.0;
    for (int i = 0; i < m; ++i) {
      Vn[i] = A.VH[i] + vxc_of(A.n[i], xc);
      d = std::max(d, std::fabs(Vn[i] - Vs[i]));
      big = std::max(big, std::fabs(Vn[i]));
    }
    if (d <= 1e-12 * big) {
      A.iters = it;
      return true;
    }
    for (int i = 0; i < m; ++i) Vs[i] += 0.3 * (Vn[i] - Vs[i]);
  }
  return false;
}

// internal energy K_e + int n Vion + (1/2) int n V_H + int n eps_xc
double energy(const Radial& g, const std::vector<double>& n, const std::vector<double>& Vion, double kT, bool xc) {
  const int m = g.size();
  const double cn = cn_of(kT);
  std::vector<double> VH, Q;
  hartree(g, n, VH, Q);
  double K = 0.0, Ei = 0.0, Eh = 0.0, Ex = 0.0;
  const double p0c = (2.0 / 3.0) * kT * (std::sqrt(2.0) / (PI * PI)) * std::pow(kT, 1.5);
  for (int i = 0; i < m; ++i) {
    const double w4 = g.w[i] * 4.0 * PI * g.r[i] * g.r[i];
    const double eta = host_fd_inverse_p12(n[i] / cn);
    K += w4 * p0c * host_fd(2, eta);
    Ei += w4 * n[i] * Vion[i];
    Eh += w4 * n[i] * VH[i];
    Ex += w4 * n[i] * exc_of(n[i], xc);
  }
  return 1.5 * K + Ei + 0.5 * Eh + Ex;
}

}  // namespace

extern "C" arche_status arche_aa_pseudopotential(const arche_aa_params* p, double dq, int32_t n_q, double* table_out,
                                                 arche_aa_result* out) {
  if (!p || !table_out || !out || n_q < 1 || !(dq > 0.0) || !(p->Z > 0.0) || !(p->rho_ion > 0.0) ||
      !(p->kT > 0.0) || !(p->r_cut_frac > 0.0 && p->r_cut_frac < 1.0) || p->n_radial < 101 ||
      (p->xc != ARCHE_XC_NONE && p->xc != ARCHE_XC_LDA))
    return ARCHE_EINVAL;
  const bool xc = p->xc == ARCHE_XC_LDA;
  const double Z = p->Z, kT = p->kT, cn = cn_of(kT);
  const double r_ws = std::cbrt(3.0 / (4.0 * PI * p->rho_ion));
  Radial g(r_ws, p->n_radial);
  const int m = g.size();
  std::vector<double> coul(m);
  for (int i = 0; i < m; ++i) coul[i] = -Z / g.r[i];
  Atom A;
  if (!solve_atom(g, Z, kT, coul, xc, A)) return ARCHE_ENOCONV;
  // r_cut on the first node at or beyond r_cut_frac r_ws
  const int ic = (int)(std::lower_bound(g.r.begin(), g.r.end(), p->r_cut_frac * r_ws) - g.r.begin());
  if (ic <= 0 || ic >= m - 1) return ARCHE_EINVAL;
  const double rc = g.r[ic];
  // n'(r_cut) from the TF relation: n' = dn/deta eta', eta' = -(Z/r^2 - Q/r^2 + v_xc'(n) n')/kT
  const double nc = A.n[ic];
  const double eta_c = host_fd_inverse_p12(nc / cn);
  const double dndeta = cn * 0.5 * host_fd(0, eta_c);
  double dvxc = 0.0;
  if (xc) {
    const double h = 1e-6 * nc;
    dvxc = (vxc_of(nc + h, xc) - vxc_of(nc - h, xc)) / (2.0 * h);
  }
  const double slope = -dndeta * (Z / (rc * rc) - A.Q[ic] / (rc * rc)) / kT / (1.0 + dndeta * dvxc / kT);
  const double y0 = std::log(nc), y1 = slope / nc;
  // the charge inside r_cut, trapezoid with the end node at half weight
  auto wq = [&](int i) { return i < ic ? g.w[i] : (i == ic ? 0.5 * g.w[i] : 0.0); };
  double q_true = 0.0;
  for (int i = 0; i <= ic; ++i) q_true += wq(i) * 4.0 * PI * g.r[i] * g.r[i] * A.n[i];
  auto ab = [&](double c, double* a, double* b) {
    *b = (y1 - 4.0 * c * rc * rc * rc) / (2.0 * rc);
    *a = y0 - *b * rc * rc - c * rc * rc * rc * rc;
  };
  auto charge = [&](double c) {
    double a, b, s = 0.0;
    ab(c, &a, &b);
    for (int i = 0; i <= ic; ++i) {
      const double r = g.r[i];
      s += wq(i) * 4.0 * PI * r * r * std::exp(a + b * r * r + c * r * r * r * r);
    }
    return s - q_true;
  };
  // the exponent is y0 + y1 (r^2 - r_c^2)/(2 r_c) + c (r^2 - r_c^2)^2: the charge grows with c
  double lo = -1.0, hi = 1.0;
  for (int k = 0; k < 200 && charge(lo) > 0; ++k) lo *= 2.0;
  for (int k = 0; k < 200 && charge(hi) < 0; ++k) hi *= 2.0;
  double c = 0.0;
  for (int k = 0; k < 400; ++k) {
    c = 0.5 * (lo + hi);
    if (charge(c) > 0)
      hi = c;
    else
      lo = c;
    if (hi - lo <= 1e-15 * std::max(1.0, std::fabs(c))) break;
  }
  c = 0.5 * (lo + hi);
  double a, b;
  ab(c, &a, &b);
  std::vector<double> np(m), Vp(m), dV(m), VHp, Qp;
  for (int i = 0; i < m; ++i) {
    const double r = g.r[i];
    np[i] = r <= rc ? std::exp(a + b * r * r + c * r * r * r * r) : A.n[i];
  }
  hartree(g, np, VHp, Qp);
  for (int i = 0; i < m; ++i) {
    const double r = g.r[i];
    if (r <= rc) {
      const double eta = host_fd_inverse_p12(np[i] / cn);
      Vp[i] = A.mu - kT * eta - vxc_of(np[i], xc) - VHp[i];
      dV[i] = Vp[i] + Z / r;
    } else {
      Vp[i] = -Z / r;
      dV[i] = 0.0;
    }
  }
  // D(q) = 4 pi int dV r^2 sin(2 pi q r)/(2 pi q r) dr
  for (int k = 0; k < n_q; ++k) {
    const double q = k * dq;
    double s = 0.0;
    for (int i = 0; i < m; ++i) {
      const double x = 2.0 * PI * q * g.r[i];
      const double j0 = x > 0.0 ? std::sin(x) / x : 1.0;
      s += g.w[i] * 4.0 * PI * dV[i] * g.r[i] * g.r[i] * j0;
    }
    table_out[k] = s;
  }
  out->r_ws = r_ws;
  out->r_cut = rc;
  out->mu = A.mu;
  out->a = a;
  out->b = b;
  out->c = c;
  out->iters = A.iters;
  out->dE_AA = energy(g, A.n, coul, kT, xc) - energy(g, np, Vp, kT, xc);
  return ARCHE_OK;
}
