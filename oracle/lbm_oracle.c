/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain FP64 CPU reference of the axisymmetric multiphase lattice Boltzmann
 * step of arXiv:1512.01977 (Reijers, Gelderblom, Toschi).  Written for
 * reading, not for speed: one pass over the grid per quantity, in the order
 * the paper introduces the quantities, with every field extended to ghost
 * nodes by an explicit accessor.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark call it; it shares no code with the HIP
 * library.
 *
 * Readings of passages the paper leaves open (each is a flag or a stated
 * choice here):
 *  - Force application: the exact-difference method named in Sec. 2.3 by
 *    default; Guo's term printed in Sec. 2.1 as the alternative (flag
 *    `forcing`), with its garbled second term read as (c_i.u)(c_i.F)/c_s^4 and
 *    BGK relaxing toward E(rho, u) at the physical velocity u = (j + F/2)/rho.
 *  - h_i (Sec. 2.2) belongs at the link midpoint (x + c_i/2, t + 1/2); the
 *    paper gives no discretisation.  Default: evaluated from the fields at
 *    (x, t).  Flag source_mid = 1: the mean of h_i at the link's two ends x and
 *    x + c_i, both at time t (second order in space along the link; the half
 *    time step would need the next step's fields, an implicit scheme), with
 *    mirrored sources beyond the walls.  Both variants are pinned as
 *    functions (the moments of h_i; the link average's totals and its order
 *    of accuracy against h_i at x + c_i/2); which time level the paper meant
 *    is not fixed by any value it prints.
 *  - H_z, H_r (eq. axihz) are node scalars; the stray c_iz, c_ir factors in
 *    the printed equation are dropped, otherwise sum_i h_i would not equal
 *    -rho u_r / r as eq. (masscylinderical) requires.
 *  - H_r carries -u_r/r, matching C_r = 2 mu d/dr(u_r / r) of Sec. 2.2
 *    (flag hr_printed_sign = 1 gives the printed +u_r/r).
 *  - mu = rho nu with nu = (tau - 1/2)/3.
 *  - The velocity in h_i and in its gradients is the physical one,
 *    u = (j + F/2)/rho (Sec. 2.1).
 *  - c_s^4 in F_axis (eq. multiphasecorrections) is replaced by
 *    c_k^4 = (dP_k/drho)^2, which stays real inside the spinodal region
 *    (flag faxis_sound = 1 keeps the lattice value 1/9).  F_K keeps its
 *    discrete form, which has no sound speed in it.
 *  - d/dr [(1/r) dpsi/dr] = D_rr psi / r - D_r psi / r^2 with the paper's
 *    stencils (eq. fifthorderaccuratefinitedifference), D_rr = D_r(D_r).
 *  - Boundaries: z periodic; mid-grid specular reflection at the axis and
 *    at a free-slip wall r = nr; half-way bounce-back for a no-slip wall.
 *    Stencils see ghost rows mirrored with parity (even for rho, psi,
 *    D_z psi, u_z; odd for u_r, D_r psi; u_z odd at a no-slip wall).
 */
#include "lbm_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

/* D2Q9 velocity set and quadrature weights, Sec. 2.1. */
static const int CZ[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CR[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WGT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

#define ERR_ARG (-1)
#define ERR_EOS (-4)
#define ERR_NONFINITE (-5)

static size_t at(int nz, int k, int j) { return (size_t)j * (size_t)nz + (size_t)k; }

/* ------------------------------------------------------------------------ */
/* Equation of state, Sec. 2.3                                               */
/* ------------------------------------------------------------------------ */

/* Largest density the EOS is defined for (exclusive). */
static double eos_rho_max(const lbm_oracle_params* p) {
  if (p->eos == ORACLE_EOS_VDW) return 3.0;
  if (p->eos == ORACLE_EOS_CS) return 4.0 / p->eos_b;
  return INFINITY;
}

/* P_k and dP_k/drho at temperature T. */
static void eos_pk(const lbm_oracle_params* p, double T, double rho, double* P, double* kappa) {
  if (p->eos == ORACLE_EOS_VDW) {
    /* eq. (kupershtokvdwpressure) and its derivative, eq. (kupershtokhspeedofsound) */
    *P = p->lambda * (8.0 * rho * T / (3.0 - rho) - 3.0 * rho * rho);
    *kappa = p->lambda * (24.0 * T / ((rho - 3.0) * (rho - 3.0)) - 6.0 * rho);
  } else if (p->eos == ORACLE_EOS_CS) {
    /* Carnahan-Starling: P = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2,
     * eta = b rho / 4; d(rho g(eta))/drho = (1 + 4eta + 4eta^2 - 4eta^3 + eta^4)/(1-eta)^4. */
    double eta = p->eos_b * rho / 4.0;
    double om = 1.0 - eta;
    double num = 1.0 + eta + eta * eta - eta * eta * eta;
    double dnum = 1.0 + 4.0 * eta + 4.0 * eta * eta - 4.0 * eta * eta * eta + eta * eta * eta * eta;
    *P = p->lambda * (rho * p->eos_R * T * num / (om * om * om) - p->eos_a * rho * rho);
    *kappa = p->lambda * (p->eos_R * T * dnum / (om * om * om * om) - 2.0 * p->eos_a * rho);
  } else {
    /* ideal gas of the lattice: P = c_s^2 rho */
    *P = rho / 3.0;
    *kappa = 1.0 / 3.0;
  }
}

int lbm_oracle_eos(const lbm_oracle_params* p, double rho, double* P, double* kappa,
                   double* psi) {
  if (!p || !P || !kappa || !psi) return ERR_ARG;
  if (!(rho > 0.0) || !(rho < eos_rho_max(p))) return ERR_EOS;
  eos_pk(p, p->T, rho, P, kappa);
  /* psi = sqrt(rho/3 - P_k), Sec. 2.3 */
  double s = rho / 3.0 - *P;
  if (p->eos == ORACLE_EOS_IDEAL) s = 0.0;
  if (s < 0.0) return ERR_EOS;
  *psi = sqrt(s);
  if (!isfinite(*P) || !isfinite(*kappa)) return ERR_NONFINITE;
  return 0;
}

/* Temperature at which kappa(rho) = 0.  kappa is affine in T for both
 * non-ideal equations of state, so two evaluations fix it. */
static double spinodal_T(const lbm_oracle_params* p, double rho) {
  double P, k0, k1;
  eos_pk(p, 0.0, rho, &P, &k0);
  eos_pk(p, 1.0, rho, &P, &k1);
  return -k0 / (k1 - k0);
}

int lbm_oracle_critical(const lbm_oracle_params* p, double* rho_c, double* T_c, double* P_c) {
  if (!p || !rho_c || !T_c || !P_c) return ERR_ARG;
  if (p->eos != ORACLE_EOS_VDW && p->eos != ORACLE_EOS_CS) return ERR_ARG;
  /* The critical point is the top of the spinodal curve T_sp(rho): golden-section search. */
  const double g = 0.5 * (sqrt(5.0) - 1.0);
  double lo = 1e-9 * eos_rho_max(p), hi = (1.0 - 1e-9) * eos_rho_max(p);
  double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo);
  double f1 = spinodal_T(p, x1), f2 = spinodal_T(p, x2);
  for (int it = 0; it < 400 && hi - lo > 1e-15 * hi; ++it) {
    if (f1 < f2) {
      lo = x1; x1 = x2; f1 = f2;
      x2 = lo + g * (hi - lo); f2 = spinodal_T(p, x2);
    } else {
      hi = x2; x2 = x1; f2 = f1;
      x1 = hi - g * (hi - lo); f1 = spinodal_T(p, x1);
    }
  }
  *rho_c = 0.5 * (lo + hi);
  *T_c = spinodal_T(p, *rho_c);
  double kap;
  eos_pk(p, *T_c, *rho_c, P_c, &kap);
  return 0;
}

/* Bisection for g(x) = 0 on [a, b] with g(a) and g(b) of opposite sign. */
static double bisect(double (*g)(const lbm_oracle_params*, double, double), const lbm_oracle_params* p,
                     double arg, double a, double b) {
  double ga = g(p, a, arg);
  for (int it = 0; it < 300; ++it) {
    double m = 0.5 * (a + b);
    if (m <= a || m >= b) break;
    double gm = g(p, m, arg);
    if ((gm < 0.0) == (ga < 0.0)) {
      a = m; ga = gm;
    } else {
      b = m;
    }
  }
  return 0.5 * (a + b);
}

static double kappa_at(const lbm_oracle_params* p, double rho, double unused) {
  (void)unused;
  double P, k;
  eos_pk(p, p->T, rho, &P, &k);
  return k;
}

static double p_minus(const lbm_oracle_params* p, double rho, double psat) {
  double P, k;
  eos_pk(p, p->T, rho, &P, &k);
  return P - psat;
}

/* Equal-area integral int_{rho_v}^{rho_l} (P - P_sat) / rho^2 drho, i.e.
 * int (P - P_sat) dv over the specific volume v = 1/rho; evaluated with
 * composite Simpson in x = ln(rho), where drho / rho^2 = dx / rho. */
static double area(const lbm_oracle_params* p, double rv, double rl, double psat) {
  const int n = 20000;
  double a = log(rv), b = log(rl), h = (b - a) / n, s = 0.0;
  for (int i = 0; i <= n; ++i) {
    double x = a + i * h, rho = exp(x);
    double w = (i == 0 || i == n) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
    s += w * p_minus(p, rho, psat) / rho;
  }
  return s * h / 3.0;
}

int lbm_oracle_coexistence(const lbm_oracle_params* p, double* rho_v, double* rho_l,
                           double* p_sat) {
  if (!p || !rho_v || !rho_l || !p_sat) return ERR_ARG;
  double rc, Tc, Pc;
  if (lbm_oracle_critical(p, &rc, &Tc, &Pc) != 0) return ERR_ARG;
  if (!(p->T > 0.0 && p->T < Tc)) return ERR_ARG;
  /* Spinodals: kappa changes sign at s1 (maximum of P) and s2 (minimum of P). */
  double rmax = eos_rho_max(p);
  const int nscan = 200000;
  double s1 = -1.0, s2 = -1.0, prev = rmax * 1e-12, kprev = kappa_at(p, prev, 0.0);
  for (int i = 1; i < nscan; ++i) {
    double r = rmax * i / nscan, k = kappa_at(p, r, 0.0);
    if (s1 < 0.0 && kprev > 0.0 && k <= 0.0) s1 = bisect(kappa_at, p, 0.0, prev, r);
    if (s1 > 0.0 && s2 < 0.0 && kprev < 0.0 && k >= 0.0) s2 = bisect(kappa_at, p, 0.0, prev, r);
    prev = r; kprev = k;
  }
  if (s1 < 0.0 || s2 < 0.0) return ERR_ARG;
  double Phi, Plo, kap;
  eos_pk(p, p->T, s1, &Phi, &kap);
  eos_pk(p, p->T, s2, &Plo, &kap);
  if (Plo < 0.0) Plo = 0.0;
  /* Bisection on P_sat: the area is positive near Plo and negative near Phi. */
  double a = Plo, b = Phi, rv = 0.0, rl = 0.0;
  for (int it = 0; it < 200; ++it) {
    double m = 0.5 * (a + b);
    if (m <= a || m >= b) break;
    rv = bisect(p_minus, p, m, rmax * 1e-14, s1);
    rl = bisect(p_minus, p, m, s2, rmax * (1.0 - 1e-14));
    if (area(p, rv, rl, m) > 0.0) a = m; else b = m;
  }
  *p_sat = 0.5 * (a + b);
  *rho_v = bisect(p_minus, p, *p_sat, rmax * 1e-14, s1);
  *rho_l = bisect(p_minus, p, *p_sat, s2, rmax * (1.0 - 1e-14));
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Lattice Boltzmann building blocks, Sec. 2.1                               */
/* ------------------------------------------------------------------------ */

void lbm_oracle_equilibrium(double rho, double uz, double ur, double feq[9]) {
  /* E_i = w_i rho [1 + (c.u)/c_s^2 + (c.u)^2/(2 c_s^4) - |u|^2/(2 c_s^2)], c_s^2 = 1/3 */
  double uu = uz * uz + ur * ur;
  for (int i = 0; i < 9; ++i) {
    double cu = CZ[i] * uz + CR[i] * ur;
    feq[i] = WGT[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

/* Node field g at (k, j) extended to ghost nodes: periodic in z, mirrored
 * across r = 0 (row -1-m is row m) and across r = nr (row nr+m is row
 * nr-1-m) with parity par_axis / par_top.  One reflection suffices for the
 * radius-2 stencils as long as nr >= 2. */
static double ext(const double* g, int nz, int nr, int k, int j, double par_axis, double par_top) {
  double s = 1.0;
  k = ((k % nz) + nz) % nz;
  if (j < 0) {
    j = -1 - j;
    s = par_axis;
  } else if (j >= nr) {
    j = 2 * nr - 1 - j;
    s = par_top;
  }
  return s * g[at(nz, k, j)];
}

/* eq. (fifthorderaccuratefinitedifference): isotropic first derivative
 *   D_a g(x) = (1/36) sum_{i=1..8} [8 g(x + c_i) - g(x + 2 c_i)] c_ia. */
static double stencil(const double* g, int nz, int nr, int k, int j, int axis, double pa, double pt) {
  double s = 0.0;
  for (int i = 1; i < 9; ++i) {
    int ca = axis == 0 ? CZ[i] : CR[i];
    if (ca == 0) continue;
    s += ca * (8.0 * ext(g, nz, nr, k + CZ[i], j + CR[i], pa, pt) -
               ext(g, nz, nr, k + 2 * CZ[i], j + 2 * CR[i], pa, pt));
  }
  return s / 36.0;
}

int lbm_oracle_derivative(const double* g, int32_t nz, int32_t nr, int32_t axis,
                          double par_axis, double par_top, double* out) {
  if (!g || !out || nz < 1 || nr < 2 || (axis != 0 && axis != 1)) return ERR_ARG;
#pragma omp parallel for
  for (int j = 0; j < nr; ++j)
    for (int k = 0; k < nz; ++k) out[at(nz, k, j)] = stencil(g, nz, nr, k, j, axis, par_axis, par_top);
  return 0;
}

static double radius(int j) { return j + 0.5; }

/* u_z mirror parity at r = nr: even at a free-slip wall, odd at a no-slip wall. */
static double top_parity_uz(const lbm_oracle_params* p) {
  return p->bc_top == ORACLE_TOP_NO_SLIP ? -1.0 : 1.0;
}

int lbm_oracle_force_psi(const lbm_oracle_params* p, const double* psi, const double* kappa,
                         double* Fz, double* Fr) {
  if (!p || !psi || !Fz || !Fr) return ERR_ARG;
  const int nz = p->nz, nr = p->nr;
  if (nz < 1 || nr < 2) return ERR_ARG;
  if (p->axisym && p->faxis_sound == 0 && !kappa) return ERR_ARG;
  size_t n = (size_t)nz * nr;
  double* dz = malloc(n * sizeof(double));
  double* dr = malloc(n * sizeof(double));
  double* drr = malloc(n * sizeof(double));
  double* drz = malloc(n * sizeof(double));
  if (!dz || !dr || !drr || !drz) {
    free(dz); free(dr); free(drr); free(drz);
    return ERR_ARG;
  }
  /* psi is even across both walls, so D_z psi is even and D_r psi odd. */
  lbm_oracle_derivative(psi, nz, nr, 0, 1.0, 1.0, dz);
  lbm_oracle_derivative(psi, nz, nr, 1, 1.0, 1.0, dr);
  lbm_oracle_derivative(dr, nz, nr, 1, -1.0, -1.0, drr);
  lbm_oracle_derivative(dz, nz, nr, 1, 1.0, 1.0, drz);
#pragma omp parallel for
  for (int j = 0; j < nr; ++j) {
    for (int k = 0; k < nz; ++k) {
      size_t x = at(nz, k, j);
      /* eq. (kupershtokhforcing) with 18/(3 dt) = 6 */
      double s2z = 0.0, s2r = 0.0, s1z = 0.0, s1r = 0.0;
      for (int i = 1; i < 9; ++i) {
        double q = ext(psi, nz, nr, k + CZ[i], j + CR[i], 1.0, 1.0);
        s2z += WGT[i] * q * q * CZ[i];
        s2r += WGT[i] * q * q * CR[i];
        s1z += WGT[i] * q * CZ[i];
        s1r += WGT[i] * q * CR[i];
      }
      double fz = 6.0 * (p->A * s2z + (1.0 - 2.0 * p->A) * psi[x] * s1z);
      double fr = 6.0 * (p->A * s2r + (1.0 - 2.0 * p->A) * psi[x] * s1r);
      if (p->axisym) {
        /* eq. (multiphasecorrections):
         * F_axis = 3 K [psi grad_c((1/r) dpsi/dr) + (6A/r) (dpsi/dr) grad_c psi],
         * K = c^4 with c the lattice or the thermodynamic sound speed. */
        double r = radius(j);
        double K = p->faxis_sound ? 1.0 / 9.0 : kappa[x] * kappa[x];
        double gz_ = drz[x] / r;
        double gr_ = drr[x] / r - dr[x] / (r * r);
        fz += 3.0 * K * (psi[x] * gz_ + 6.0 * p->A / r * dr[x] * dz[x]);
        fr += 3.0 * K * (psi[x] * gr_ + 6.0 * p->A / r * dr[x] * dr[x]);
      }
      Fz[x] = fz + p->gz;
      Fr[x] = fr;
    }
  }
  free(dz); free(dr); free(drr); free(drz);
  return 0;
}

void lbm_oracle_source(const lbm_oracle_params* p, double r, double rho, double uz, double ur,
                       double dr_uz, double dz_ur, double dr_ur, double h[9]) {
  /* eq. (axihz) with mu = rho (tau - 1/2) / 3 */
  double mu = rho * (p->tau - 0.5) / 3.0;
  double sgn = p->hr_printed_sign ? 1.0 : -1.0;
  double Hz = (mu * (dr_uz + dz_ur) - rho * ur * uz) / r;
  double Hr = (2.0 * mu * (dr_ur + sgn * ur / r) - rho * ur * ur) / r;
  for (int i = 0; i < 9; ++i)
    h[i] = WGT[i] * (-rho * ur / r + 3.0 * (CZ[i] * Hz + CR[i] * Hr));
}

void lbm_oracle_guo_source(double tau, double uz, double ur, double Fz, double Fr, double S[9]) {
  /* Sec. 2.1 with c_s^2 = 1/3: (c_i - u).F / c_s^2 + (c_i.u)(c_i.F) / c_s^4 */
  double pre = 1.0 - 0.5 / tau;
  for (int i = 0; i < 9; ++i) {
    double cu = CZ[i] * uz + CR[i] * ur;
    double cF = CZ[i] * Fz + CR[i] * Fr;
    double cmuF = (CZ[i] - uz) * Fz + (CR[i] - ur) * Fr;
    S[i] = WGT[i] * pre * (3.0 * cmuF + 9.0 * cu * cF);
  }
}

/* Mirror of direction i across a wall: (c_z, c_r) -> (c_z, -c_r). */
static int mirror_dir(int i) {
  for (int q = 0; q < 9; ++q)
    if (CZ[q] == CZ[i] && CR[q] == -CR[i]) return q;
  return i;
}

/* Source of direction i at node (k, j), which may lie one row beyond the axis or the wall:
 * there it is the source of the mirror node in the mirrored direction, since -rho u_r / r
 * and H_z are even and H_r is odd under the reflection. */
static double source_ext(const double* hn, int nz, int nr, int i, int k, int j) {
  const size_t n = (size_t)nz * nr;
  k = ((k % nz) + nz) % nz;
  if (j < 0) return hn[(size_t)mirror_dir(i) * n + at(nz, k, -1 - j)];
  if (j >= nr) return hn[(size_t)mirror_dir(i) * n + at(nz, k, 2 * nr - 1 - j)];
  return hn[(size_t)i * n + at(nz, k, j)];
}

int lbm_oracle_source_field(const lbm_oracle_params* p, const double* rho, const double* uz,
                            const double* ur, double* h) {
  if (!p || !rho || !uz || !ur || !h || p->nz < 1 || p->nr < 2) return ERR_ARG;
  const int nz = p->nz, nr = p->nr;
  const size_t n = (size_t)nz * nr;
  if (!p->axisym) {
    memset(h, 0, 9 * n * sizeof(double));
    return 0;
  }
  double* druz = malloc(n * sizeof(double));
  double* dzur = malloc(n * sizeof(double));
  double* drur = malloc(n * sizeof(double));
  double* hn = p->source_mid ? malloc(9 * n * sizeof(double)) : h;
  if (!druz || !dzur || !drur || !hn) {
    free(druz); free(dzur); free(drur);
    if (hn != h) free(hn);
    return ERR_ARG;
  }
  /* velocity derivatives for H, with the same stencil (Sec. 2.2) */
  lbm_oracle_derivative(uz, nz, nr, 1, 1.0, top_parity_uz(p), druz);
  lbm_oracle_derivative(ur, nz, nr, 0, -1.0, -1.0, dzur);
  lbm_oracle_derivative(ur, nz, nr, 1, -1.0, -1.0, drur);
#pragma omp parallel for
  for (int j = 0; j < nr; ++j)
    for (int k = 0; k < nz; ++k) {
      size_t x = at(nz, k, j);
      double hx[9];
      lbm_oracle_source(p, radius(j), rho[x], uz[x], ur[x], druz[x], dzur[x], drur[x], hx);
      for (int i = 0; i < 9; ++i) hn[(size_t)i * n + x] = hx[i];
    }
  if (p->source_mid) {
    /* Sec. 2.2: h_i at x + c_i/2, the mean over the link's two ends */
#pragma omp parallel for
    for (int j = 0; j < nr; ++j)
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < 9; ++i)
          h[(size_t)i * n + at(nz, k, j)] =
              0.5 * (source_ext(hn, nz, nr, i, k, j) + source_ext(hn, nz, nr, i, k + CZ[i], j + CR[i]));
    free(hn);
  }
  free(druz); free(dzur); free(drur);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Whole step                                                                 */
/* ------------------------------------------------------------------------ */

static int check_params(const lbm_oracle_params* p) {
  if (!p) return ERR_ARG;
  if (p->nz < 1 || p->nr < 4) return ERR_ARG;
  if (!(p->tau > 0.5)) return ERR_ARG;
  if (p->eos < ORACLE_EOS_IDEAL || p->eos > ORACLE_EOS_CS) return ERR_ARG;
  if (p->bc_top != ORACLE_TOP_FREE_SLIP && p->bc_top != ORACLE_TOP_NO_SLIP) return ERR_ARG;
  if (p->forcing != ORACLE_FORCING_EDM && p->forcing != ORACLE_FORCING_GUO) return ERR_ARG;
  if (p->source_mid != 0 && p->source_mid != 1) return ERR_ARG;
  return 0;
}

/* Density and momentum j = sum_i c_i f_i of the post-streaming populations. */
static void moments0(int nz, int nr, const double* f, double* rho, double* jz, double* jr) {
  size_t n = (size_t)nz * nr;
#pragma omp parallel for
  for (int j = 0; j < nr; ++j) {
    for (int k = 0; k < nz; ++k) {
      size_t x = at(nz, k, j);
      double s = 0.0, sz = 0.0, sr = 0.0;
      for (int i = 0; i < 9; ++i) {
        double fi = f[i * n + x];
        s += fi;
        sz += CZ[i] * fi;
        sr += CR[i] * fi;
      }
      rho[x] = s;
      jz[x] = sz;
      jr[x] = sr;
    }
  }
}

/* Pseudopotential and kappa on the grid; returns the first error. */
static int eos_field(const lbm_oracle_params* p, const double* rho, double* psi, double* kappa) {
  size_t n = (size_t)p->nz * p->nr;
  int err = 0;
  for (size_t x = 0; x < n; ++x) {
    double P;
    int e = lbm_oracle_eos(p, rho[x], &P, &kappa[x], &psi[x]);
    if (e && !err) err = e;
  }
  return err;
}

typedef struct {
  double *rho, *jz, *jr, *psi, *kappa, *Fz, *Fr, *uz, *ur;
} fields;

static void fields_free(fields* w) {
  free(w->rho); free(w->jz); free(w->jr); free(w->psi); free(w->kappa);
  free(w->Fz); free(w->Fr); free(w->uz); free(w->ur);
}

static int fields_alloc(fields* w, size_t n) {
  memset(w, 0, sizeof(*w));
  w->rho = malloc(n * sizeof(double));
  w->jz = malloc(n * sizeof(double));
  w->jr = malloc(n * sizeof(double));
  w->psi = malloc(n * sizeof(double));
  w->kappa = malloc(n * sizeof(double));
  w->Fz = malloc(n * sizeof(double));
  w->Fr = malloc(n * sizeof(double));
  w->uz = malloc(n * sizeof(double));
  w->ur = malloc(n * sizeof(double));
  if (!w->rho || !w->jz || !w->jr || !w->psi || !w->kappa || !w->Fz || !w->Fr || !w->uz || !w->ur) {
    fields_free(w);
    return ERR_ARG;
  }
  return 0;
}

/* rho, j, psi, F and the physical velocity of the state f. */
static int macro(const lbm_oracle_params* p, const double* f, fields* w) {
  const int nz = p->nz, nr = p->nr;
  size_t n = (size_t)nz * nr;
  moments0(nz, nr, f, w->rho, w->jz, w->jr);
  int e = eos_field(p, w->rho, w->psi, w->kappa);
  if (e) return e;
  e = lbm_oracle_force_psi(p, w->psi, w->kappa, w->Fz, w->Fr);
  if (e) return e;
  for (size_t x = 0; x < n; ++x) {
    /* u = F/(2 rho) + j/rho, Sec. 2.1 */
    w->uz[x] = (w->jz[x] + 0.5 * w->Fz[x]) / w->rho[x];
    w->ur[x] = (w->jr[x] + 0.5 * w->Fr[x]) / w->rho[x];
  }
  return 0;
}

/* One time step: collide every node into fs, then stream fs back into f.  hs: [9][n]
 * scratch for the source field. */
static int one_step(const lbm_oracle_params* p, double* f, double* fs, fields* w, double* hs) {
  const int nz = p->nz, nr = p->nr;
  const size_t n = (size_t)nz * nr;
  int e = macro(p, f, w);
  if (e) return e;
  e = lbm_oracle_source_field(p, w->rho, w->uz, w->ur, hs);
  if (e) return e;
  const double omega = 1.0 / p->tau;
#pragma omp parallel for
  for (int j = 0; j < nr; ++j) {
    for (int k = 0; k < nz; ++k) {
      size_t x = at(nz, k, j);
      double rho = w->rho[x];
      double ubz = w->jz[x] / rho, ubr = w->jr[x] / rho;
      double e0[9], e1[9], h[9];
      for (int i = 0; i < 9; ++i) h[i] = hs[(size_t)i * n + x];
      if (p->forcing == ORACLE_FORCING_EDM) {
        /* exact-difference method: Delta f_i = E_i(rho, u_b + F dt/rho) - E_i(rho, u_b) */
        lbm_oracle_equilibrium(rho, ubz, ubr, e0);
        lbm_oracle_equilibrium(rho, ubz + w->Fz[x] / rho, ubr + w->Fr[x] / rho, e1);
        for (int i = 0; i < 9; ++i) {
          double fi = f[i * n + x];
          /* eq. (lbm) with the axisymmetric source of Sec. 2.2 */
          fs[i * n + x] = fi + omega * (e0[i] - fi) + (e1[i] - e0[i]) + h[i];
        }
      } else {
        /* Guo (Sec. 2.1): BGK toward E(rho, u) at the physical velocity, plus S_i */
        lbm_oracle_equilibrium(rho, w->uz[x], w->ur[x], e0);
        lbm_oracle_guo_source(p->tau, w->uz[x], w->ur[x], w->Fz[x], w->Fr[x], e1);
        for (int i = 0; i < 9; ++i) {
          double fi = f[i * n + x];
          fs[i * n + x] = fi + omega * (e0[i] - fi) + e1[i] + h[i];
        }
      }
    }
  }
  /* Pull streaming f_i(x, t+1) = f*_i(x - c_i, t) with the wall maps. */
#pragma omp parallel for
  for (int j = 0; j < nr; ++j) {
    for (int k = 0; k < nz; ++k) {
      for (int i = 0; i < 9; ++i) {
        int sk = k - CZ[i], sj = j - CR[i], si = i;
        if (sj < 0) {
          /* mid-grid specular reflection at the axis: (c_z, -1) -> (c_z, +1) */
          sj = 0;
          for (int q = 0; q < 9; ++q)
            if (CZ[q] == CZ[i] && CR[q] == -CR[i]) si = q;
        } else if (sj >= nr) {
          sj = nr - 1;
          if (p->bc_top == ORACLE_TOP_NO_SLIP) {
            /* half-way bounce-back: (c_z, +1) leaves and comes back as (-c_z, -1) */
            sk = k;
            for (int q = 0; q < 9; ++q)
              if (CZ[q] == -CZ[i] && CR[q] == -CR[i]) si = q;
          } else {
            /* mid-grid specular reflection: (c_z, +1) -> (c_z, -1) */
            for (int q = 0; q < 9; ++q)
              if (CZ[q] == CZ[i] && CR[q] == -CR[i]) si = q;
          }
        }
        sk = ((sk % nz) + nz) % nz;
        f[(size_t)i * n + at(nz, k, j)] = fs[(size_t)si * n + at(nz, sk, sj)];
      }
    }
  }
  for (size_t x = 0; x < 9 * n; ++x)
    if (!isfinite(f[x])) return ERR_NONFINITE;
  return 0;
}

int lbm_oracle_init(const lbm_oracle_params* p, const double* rho0, const double* uz0,
                    const double* ur0, double* f) {
  int e = check_params(p);
  if (e) return e;
  if (!rho0 || !f) return ERR_ARG;
  size_t n = (size_t)p->nz * p->nr;
  for (size_t x = 0; x < n; ++x) {
    double P, kap, psi;
    e = lbm_oracle_eos(p, rho0[x], &P, &kap, &psi);
    if (e) return e;
    double feq[9];
    lbm_oracle_equilibrium(rho0[x], uz0 ? uz0[x] : 0.0, ur0 ? ur0[x] : 0.0, feq);
    for (int i = 0; i < 9; ++i) f[i * n + x] = feq[i];
  }
  return 0;
}

int lbm_oracle_step(const lbm_oracle_params* p, double* f, int64_t nsteps) {
  int e = check_params(p);
  if (e) return e;
  if (!f || nsteps < 0) return ERR_ARG;
  size_t n = (size_t)p->nz * p->nr;
  fields w;
  if (fields_alloc(&w, n)) return ERR_ARG;
  double* fs = malloc(9 * n * sizeof(double));
  double* hs = malloc(9 * n * sizeof(double));
  if (!fs || !hs) e = ERR_ARG;
  for (int64_t s = 0; s < nsteps && !e; ++s) e = one_step(p, f, fs, &w, hs);
  free(fs); free(hs);
  fields_free(&w);
  return e;
}

int lbm_oracle_moments(const lbm_oracle_params* p, const double* f, double* rho, double* uz,
                       double* ur) {
  int e = check_params(p);
  if (e) return e;
  if (!f || !rho || !uz || !ur) return ERR_ARG;
  size_t n = (size_t)p->nz * p->nr;
  fields w;
  if (fields_alloc(&w, n)) return ERR_ARG;
  e = macro(p, f, &w);
  if (!e) {
    memcpy(rho, w.rho, n * sizeof(double));
    memcpy(uz, w.uz, n * sizeof(double));
    memcpy(ur, w.ur, n * sizeof(double));
  }
  fields_free(&w);
  return e;
}

int lbm_oracle_mass(const lbm_oracle_params* p, const double* f, double* mass) {
  int e = check_params(p);
  if (e) return e;
  if (!f || !mass) return ERR_ARG;
  const int nz = p->nz, nr = p->nr;
  size_t n = (size_t)nz * nr;
  double s = 0.0;
  for (int j = 0; j < nr; ++j)
    for (int k = 0; k < nz; ++k) {
      double rho = 0.0;
      for (int i = 0; i < 9; ++i) rho += f[i * n + at(nz, k, j)];
      s += 2.0 * M_PI * radius(j) * rho;
    }
  *mass = s;
  return 0;
}

int lbm_oracle_laplace(const lbm_oracle_params* p, const double* f, double zc, double r_in,
                       double r_out, double* dp) {
  int e = check_params(p);
  if (e) return e;
  if (!f || !dp) return ERR_ARG;
  const int nz = p->nz, nr = p->nr;
  size_t n = (size_t)nz * nr;
  double sin_ = 0.0, sout = 0.0;
  long cin = 0, cout = 0;
  for (int j = 0; j < nr; ++j)
    for (int k = 0; k < nz; ++k) {
      double rho = 0.0;
      for (int i = 0; i < 9; ++i) rho += f[i * n + at(nz, k, j)];
      double P, kap;
      eos_pk(p, p->T, rho, &P, &kap);
      double d = sqrt((k - zc) * (k - zc) + radius(j) * radius(j));
      if (d < r_in) { sin_ += P; ++cin; }
      if (d > r_out) { sout += P; ++cout; }
    }
  if (cin == 0 || cout == 0) return ERR_ARG;
  *dp = sin_ / cin - sout / cout;
  return 0;
}

/* Sec. 3.2 tracks the oscillating drop by where its interface crosses the symmetry axis.
 * Along the axis row (j = 0) from column k0 = floor(zc) towards +z: the first k >= k0
 * whose next node has rho_{k+1} <= thr, and the linear interpolation of rho = thr between
 * the two nodes, z = k + (rho_k - thr) / (rho_k - rho_{k+1}).  No such k before the last
 * column gives NaN. */
int lbm_oracle_axis_interface(const lbm_oracle_params* p, const double* f, double zc, double thr,
                              double* z) {
  int e = check_params(p);
  if (e) return e;
  if (!f || !z || !(zc >= 0.0) || !(zc < p->nz)) return ERR_ARG;
  const int nz = p->nz;
  const size_t n = (size_t)nz * p->nr;
  const int k0 = (int)floor(zc);
  *z = NAN;
  for (int k = k0; k + 1 < nz; ++k) {
    double rk = 0.0, rn = 0.0;
    for (int i = 0; i < 9; ++i) {
      rk += f[i * n + at(nz, k, 0)];
      rn += f[i * n + at(nz, k + 1, 0)];
    }
    if (rn <= thr) {
      *z = k + (rk - thr) / (rk - rn);
      break;
    }
  }
  return 0;
}

int lbm_oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void lbm_oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
