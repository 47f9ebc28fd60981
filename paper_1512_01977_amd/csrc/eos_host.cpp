// Host-side equation-of-state helpers of the library: critical point and Maxwell
// coexistence, used to lay out initial conditions and to convert T/T_c into T.
// They are not on the time-stepping path (which evaluates the EOS in its kernels).
#include <cmath>

#include "lbm_axi.h"
#include "lbm_axi_internal.h"

namespace lbm {

namespace {

// P_k and dP_k/drho at temperature T (Sec. 2.3 for vdW; Carnahan-Starling for CS).
void pk_host(const lbm_axi_params& p, double T, double rho, double* P, double* dP) {
  switch (p.eos) {
    case LBM_EOS_VDW: {
      const double d = 3.0 - rho;
      *P = p.lambda * (8.0 * rho * T / d - 3.0 * rho * rho);
      *dP = p.lambda * (24.0 * T / (d * d) - 6.0 * rho);
      return;
    }
    case LBM_EOS_CS: {
      const double e = 0.25 * p.eos_b * rho, m = 1.0 - e;
      const double m3 = m * m * m;
      *P = p.lambda * (p.eos_R * T * rho * (1.0 + e * (1.0 + e * (1.0 - e))) / m3 - p.eos_a * rho * rho);
      *dP = p.lambda * (p.eos_R * T * (1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)))) / (m3 * m) -
                        2.0 * p.eos_a * rho);
      return;
    }
    default:
      *P = rho / 3.0;
      *dP = 1.0 / 3.0;
  }
}

double P_at(const lbm_axi_params& p, double T, double rho) {
  double P, d;
  pk_host(p, T, rho, &P, &d);
  return P;
}

double dP_at(const lbm_axi_params& p, double T, double rho) {
  double P, d;
  pk_host(p, T, rho, &P, &d);
  return d;
}

double rho_limit(const lbm_axi_params& p) {
  return p.eos == LBM_EOS_VDW ? 3.0 : 4.0 / p.eos_b;
}

// Root of g on [lo, hi] given a sign change, by bisection to full precision.
template <class G>
double root(G g, double lo, double hi) {
  double glo = g(lo);
  for (int i = 0; i < 400; ++i) {
    const double m = 0.5 * (lo + hi);
    if (!(m > lo && m < hi)) break;
    const double gm = g(m);
    if ((gm < 0.0) == (glo < 0.0)) {
      lo = m;
      glo = gm;
    } else {
      hi = m;
    }
  }
  return 0.5 * (lo + hi);
}

// integral of dP/drho / rho over [r0, r1] (chemical-potential difference at fixed T),
// composite 5-point Gauss-Legendre in x = ln(rho) where drho/rho = dx.
double mu_diff(const lbm_axi_params& p, double T, double r0, double r1) {
  static const double xg[5] = {-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831,
                               0.9061798459386640};
  static const double wg[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                               0.4786286704993665, 0.2369268850561891};
  const int nsub = 400;
  const double a = std::log(r0), b = std::log(r1), h = (b - a) / nsub;
  double s = 0.0;
  for (int q = 0; q < nsub; ++q) {
    const double c = a + (q + 0.5) * h;
    for (int g = 0; g < 5; ++g) s += wg[g] * dP_at(p, T, std::exp(c + 0.5 * h * xg[g]));
  }
  return 0.5 * h * s;
}

}  // namespace

double eos_psi(const lbm_axi_params& p, double rho) {
  if (p.eos == LBM_EOS_IDEAL) return 0.0;
  const double s = rho / 3.0 - P_at(p, p.T, rho);
  return s > 0.0 ? std::sqrt(s) : 0.0;
}

lbm_status eos_critical(const lbm_axi_params& p, double* rho_c, double* T_c, double* P_c) {
  if (p.eos == LBM_EOS_VDW) {
    // The reduced vdW EOS has its critical point at rho = T = 1, where P_k = lambda.
    *rho_c = 1.0;
    *T_c = 1.0;
    *P_c = P_at(p, 1.0, 1.0);
    return LBM_OK;
  }
  if (p.eos != LBM_EOS_CS || !(p.eos_b > 0.0) || !(p.eos_a > 0.0) || !(p.eos_R > 0.0))
    return LBM_ERR_ARG;
  // Spinodal temperature T_sp(e) = (8a/(bR)) e (1-e)^4 / q(e), q = 1+4e+4e^2-4e^3+e^4;
  // the critical packing fraction maximises it: 1/e - 4/(1-e) - q'/q = 0.
  auto dlog = [](double e) {
    const double q = 1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)));
    const double dq = 4.0 + e * (8.0 + e * (-12.0 + 4.0 * e));
    return 1.0 / e - 4.0 / (1.0 - e) - dq / q;
  };
  const double ec = root(dlog, 0.01, 0.5);
  const double qc = 1.0 + ec * (4.0 + ec * (4.0 + ec * (-4.0 + ec)));
  const double m = 1.0 - ec;
  *rho_c = 4.0 * ec / p.eos_b;
  *T_c = 8.0 * p.eos_a / (p.eos_b * p.eos_R) * ec * m * m * m * m / qc;
  *P_c = P_at(p, *T_c, *rho_c);
  return LBM_OK;
}

lbm_status eos_coexistence(const lbm_axi_params& p, double* rho_v, double* rho_l, double* p_sat) {
  double rc, Tc, Pc;
  lbm_status s = eos_critical(p, &rc, &Tc, &Pc);
  if (s != LBM_OK) return s;
  const double T = p.T;
  if (!(T > 0.0 && T < Tc)) return LBM_ERR_ARG;
  const double rmax = rho_limit(p);
  // Spinodals: the zeros of dP/drho on either side of the critical density.
  auto kap = [&](double r) { return dP_at(p, T, r); };
  double lo = rc, hi = rc;
  while (kap(lo) < 0.0 && lo > 1e-300) lo *= 0.5;
  while (kap(hi) < 0.0 && hi < rmax) hi = 0.5 * (hi + rmax);
  if (kap(rc) >= 0.0) return LBM_ERR_ARG;
  const double s1 = root(kap, lo, rc), s2 = root(kap, rc, hi);
  // For a vapour density rv below s1, the liquid branch density of equal pressure, then
  // the equal-chemical-potential condition as a function of rv.
  auto liquid_of = [&](double rv) {
    const double Pv = P_at(p, T, rv);
    return root([&](double r) { return P_at(p, T, r) - Pv; }, s2, rmax * (1.0 - 1e-15));
  };
  const double Pmin = P_at(p, T, s2);
  // lowest admissible vapour density: pressure above both 0 and the local minimum of P
  double rv_lo = s1 * 1e-12;
  if (Pmin > 0.0) rv_lo = root([&](double r) { return P_at(p, T, r) - Pmin; }, rv_lo, s1);
  auto g = [&](double rv) { return mu_diff(p, T, rv, liquid_of(rv)); };
  double a = rv_lo * (1.0 + 1e-12), b = s1 * (1.0 - 1e-12);
  double ga = g(a);
  for (int i = 0; i < 200; ++i) {
    const double m = 0.5 * (a + b);
    if (!(m > a && m < b)) break;
    const double gm = g(m);
    if ((gm < 0.0) == (ga < 0.0)) {
      a = m;
      ga = gm;
    } else {
      b = m;
    }
  }
  *rho_v = 0.5 * (a + b);
  *rho_l = liquid_of(*rho_v);
  *p_sat = P_at(p, T, *rho_v);
  return LBM_OK;
}

}  // namespace lbm
