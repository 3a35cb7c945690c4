/*
 * Oracle (test infrastructure only): complete Fermi-Dirac integrals by direct
 * quadrature of their definition.
 *
 *   I_j(x) = integral_0^inf t^j / (exp(t - x) + 1) dt,   j in {-1/2, 1/2, 3/2}
 *
 * (paper, Sec. 2.2, the definition given with the Thomas-Fermi density
 * equation SCF1).  Only tests, the smoke check and the CPU baseline may call
 * this code; the product path never links it.
 *
 * Method, chosen to be plainly checkable rather than fast:
 *   - substitute t = u^2 so the integrand 2 u^(2j+1) / (exp(u^2 - x) + 1) is
 *     smooth at the origin for all three orders;
 *   - integrate t over [t_lo, t_hi] with t_lo = max(0, x - 40) and
 *     t_hi = max(x, 0) + 45; outside that range the Fermi factor differs from
 *     1 (below) or 0 (above) by less than exp(-40), which is below double
 *     rounding relative to the result;
 *   - the part [0, t_lo] where the Fermi factor is 1 to within exp(-40) is
 *     integrated exactly: t_lo^(j+1) / (j+1);
 *   - [t_lo, t_hi] is cut into panels at t = x + s for a fixed list of s
 *     (dense near the Fermi edge s = 0, where the integrand varies fastest)
 *     and at a fixed list of absolute t (for x <= 0, where no edge lies in
 *     range); each panel gets an n-point Gauss-Legendre rule in u.
 *
 * The Gauss-Legendre nodes/weights on [-1, 1] are passed in by the caller.
 * Each x is independent; the loop over x is parallel and per-x arithmetic
 * does not depend on the thread count.
 */
#include <math.h>
#include <stddef.h>

static const double S_EDGE[] = {-40.0, -30.0, -24.0, -19.0, -15.0, -12.0, -9.5, -7.5, -6.0,
                                -4.5,  -3.5,  -2.5,  -1.5,  -0.75, 0.0,   0.75, 1.5,  2.5,
                                3.5,   4.5,   6.0,   7.5,   9.5,   12.0,  15.0, 19.0, 24.0,
                                30.0,  37.0};
static const double T_ABS[] = {0.25, 0.75, 1.5, 2.5, 3.5, 5.0, 7.0, 9.5, 12.5, 16.0, 20.0, 25.0, 31.0, 38.0};

#define NS ((int)(sizeof(S_EDGE) / sizeof(S_EDGE[0])))
#define NT ((int)(sizeof(T_ABS) / sizeof(T_ABS[0])))

static void sort_small(double *a, int n) {
  for (int i = 1; i < n; ++i) {
    double v = a[i];
    int k = i - 1;
    while (k >= 0 && a[k] > v) { a[k + 1] = a[k]; --k; }
    a[k + 1] = v;
  }
}

/* 1/(exp(s)+1) without overflow */
static double fermi(double s) {
  if (s > 0.0) { double e = exp(-s); return e / (1.0 + e); }
  return 1.0 / (exp(s) + 1.0);
}

static void fd_one(double x, int ng, const double *gx, const double *gw,
                   double *out_m12, double *out_p12, double *out_p32) {
  double t_lo = x - 40.0 > 0.0 ? x - 40.0 : 0.0;
  double t_hi = (x > 0.0 ? x : 0.0) + 45.0;
  double b[2 + NS + NT];
  int nb = 0;
  b[nb++] = t_lo;
  b[nb++] = t_hi;
  for (int i = 0; i < NS; ++i) {
    double t = x + S_EDGE[i];
    if (t > t_lo && t < t_hi) b[nb++] = t;
  }
  for (int i = 0; i < NT; ++i) {
    double t = T_ABS[i];
    if (t > t_lo && t < t_hi) b[nb++] = t;
  }
  sort_small(b, nb);
  /* merge boundaries closer than 1e-3 in t; the end point t_hi always stays */
  double c[2 + NS + NT];
  int nc = 0;
  c[nc++] = b[0];
  for (int i = 1; i < nb; ++i) {
    if (b[i] - c[nc - 1] > 1e-3) c[nc++] = b[i];
    else if (i == nb - 1) c[nc - 1] = b[i];
  }
  /* analytic bulk [0, t_lo] */
  double sm12 = 0.0, sp12 = 0.0, sp32 = 0.0;
  if (t_lo > 0.0) {
    double r = sqrt(t_lo);
    sm12 = 2.0 * r;                  /* t^(1/2) / (1/2) */
    sp12 = t_lo * r / 1.5;           /* t^(3/2) / (3/2) */
    sp32 = t_lo * t_lo * r / 2.5;    /* t^(5/2) / (5/2) */
  }
  double am12 = 0.0, ap12 = 0.0, ap32 = 0.0;
  for (int p = 0; p + 1 < nc; ++p) {
    double ua = sqrt(c[p]), ub = sqrt(c[p + 1]);
    double h = 0.5 * (ub - ua), m = 0.5 * (ub + ua);
    double qm12 = 0.0, qp12 = 0.0, qp32 = 0.0;
    for (int q = 0; q < ng; ++q) {
      double u = m + h * gx[q];
      double u2 = u * u;
      double f = 2.0 * gw[q] * fermi(u2 - x);
      qm12 += f;            /* 2 u^0 */
      qp12 += f * u2;       /* 2 u^2 */
      qp32 += f * u2 * u2;  /* 2 u^4 */
    }
    am12 += h * qm12;
    ap12 += h * qp12;
    ap32 += h * qp32;
  }
  *out_m12 = sm12 + am12;
  *out_p12 = sp12 + ap12;
  *out_p32 = sp32 + ap32;
}

/* I_{-1/2}, I_{1/2}, I_{3/2} for each x[i]; any output pointer may be NULL. */
void oracle_fd_eval(ptrdiff_t n, const double *x, int ng, const double *gx, const double *gw,
                    double *im12, double *ip12, double *ip32) {
#pragma omp parallel for schedule(static) if (n > 2048)
  for (ptrdiff_t i = 0; i < n; ++i) {
    double a, b, c;
    fd_one(x[i], ng, gx, gw, &a, &b, &c);
    if (im12) im12[i] = a;
    if (ip12) ip12[i] = b;
    if (ip32) ip32[i] = c;
  }
}
