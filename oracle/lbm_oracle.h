/*
 * lbm_oracle.h -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, FP64 CPU implementation of the axisymmetric pseudopotential
 * lattice Boltzmann step of Reijers, Gelderblom and Toschi, "Axisymmetric
 * multiphase lattice Boltzmann method for generic equations of state"
 * (arXiv:1512.01977).  It exists only to check the HIP path: the tests, the
 * smoke check and the CPU-baseline leg of the benchmark are its only callers.
 * It shares no source with the HIP library.
 *
 * Grid: node (k, j) sits at z = k (k = 0..nz-1) and r = j + 1/2
 * (j = 0..nr-1); the symmetry axis r = 0 lies half-way between the ghost row
 * j = -1 and the first row (mid-grid, Sec. 3.1).  Node fields are [nr][nz]
 * arrays with k fastest.  The distribution is f[9][nr][nz].
 *
 * D2Q9 directions (c_z, c_r), Sec. 2.1:
 *   0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
 *
 * Every entry point returns 0 on success or a negative code:
 *   -1 bad argument, -4 equation-of-state domain left (rho <= 0, or
 *   rho/3 - P_k < 0 so that psi is not real), -5 non-finite value.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_EOS_IDEAL = 0, ORACLE_EOS_VDW = 1, ORACLE_EOS_CS = 2 };
enum { ORACLE_TOP_FREE_SLIP = 0, ORACLE_TOP_NO_SLIP = 1 };
enum { ORACLE_FORCING_EDM = 0, ORACLE_FORCING_GUO = 1 };

typedef struct {
  int32_t nz, nr;          /* nz >= 1, nr >= 4 */
  double tau;              /* BGK relaxation time, > 1/2 */
  int32_t eos;             /* ORACLE_EOS_* */
  double T;                /* absolute temperature of the EOS */
  double eos_a, eos_b, eos_R; /* Carnahan-Starling a, b, R */
  double lambda;           /* pressure scale multiplying P_k (vdW and CS) */
  double A;                /* Kupershtokh mixing parameter */
  int32_t axisym;          /* 1: axisymmetric source terms and force correction */
  int32_t faxis_sound;     /* 0: c^4 in F_axis is (dP_k/drho)^2; 1: c_s^4 = 1/9 */
  int32_t bc_top;          /* ORACLE_TOP_* at r = nr */
  int32_t hr_printed_sign; /* 0: H_r with -u_r/r (follows C_r); 1: as printed, +u_r/r */
  double gz;               /* uniform body-force density along z */
  int32_t forcing;         /* ORACLE_FORCING_EDM (Sec. 2.3) or ORACLE_FORCING_GUO (Sec. 2.1) */
  int32_t source_mid;      /* 0: h_i at the node (x, t); 1: h_i at the link midpoint x + c_i/2,
                              as the mean of h_i at the link's two ends (Sec. 2.2) */
} lbm_oracle_params;

/* Equation of state at density rho: pressure P_k, kappa = dP_k/drho and the
 * pseudopotential psi = sqrt(rho/3 - P_k).  Returns -4 outside its domain. */
int lbm_oracle_eos(const lbm_oracle_params* p, double rho, double* P, double* kappa,
                   double* psi);

/* Critical point (rho_c, T_c, P_c) of the EOS kind/coefficients in p (T ignored). */
int lbm_oracle_critical(const lbm_oracle_params* p, double* rho_c, double* T_c, double* P_c);

/* Maxwell equal-area coexistence densities and saturation pressure at p->T. */
int lbm_oracle_coexistence(const lbm_oracle_params* p, double* rho_v, double* rho_l,
                           double* p_sat);

/* Second-order equilibrium E_i(rho, u), Sec. 2.1 with c_s^2 = 1/3. */
void lbm_oracle_equilibrium(double rho, double uz, double ur, double feq[9]);

/* Isotropic fifth-order first derivative (axis 0: d/dz, 1: d/dr) of a node
 * field g, extended periodically in z and mirrored with the given parities
 * (+1 or -1) across r = 0 and r = nr. */
int lbm_oracle_derivative(const double* g, int32_t nz, int32_t nr, int32_t axis,
                          double par_axis, double par_top, double* out);

/* Multiphase force F = F_K (+ F_axis if axisym) + (gz, 0) from a psi field and
 * a kappa field (kappa only read when axisym and faxis_sound == 0). */
int lbm_oracle_force_psi(const lbm_oracle_params* p, const double* psi, const double* kappa,
                         double* Fz, double* Fr);

/* Axisymmetric source h_i at one node of radius r, from rho, the physical
 * velocity u and the three velocity derivatives it needs. */
void lbm_oracle_source(const lbm_oracle_params* p, double r, double rho, double uz, double ur,
                       double dr_uz, double dz_ur, double dr_ur, double h[9]);

/* The source h_i of every node that one step adds, as [9][nr][nz], from node fields
 * rho and the physical velocity u (the velocity derivatives are taken here with the
 * stencil of eq. fifthorderaccuratefinitedifference).  source_mid = 0: h_i(x) of
 * eq. (axihz) at the node.  source_mid = 1: the evolution equation of Sec. 2.2 evaluates
 * h_i half-way along the link, at x + c_i/2; here the mean of h_i at x and at x + c_i,
 * both at time t.  Beyond the axis or the wall, h_i(x + c_i) is that of the mirror node
 * in the mirrored direction (-rho u_r/r and H_z even, H_r odd).  All zeros in 2-D mode. */
int lbm_oracle_source_field(const lbm_oracle_params* p, const double* rho, const double* uz,
                            const double* ur, double* h);

/* Guo's forcing term S_i of Sec. 2.1 at one node: w_i (1 - 1/(2 tau)) [3 (c_i - u).F +
 * 9 (c_i.u)(c_i.F)], u the physical velocity (the printed second term is read as
 * (c_i.u)(c_i.F)/c_s^4). */
void lbm_oracle_guo_source(double tau, double uz, double ur, double Fz, double Fr, double S[9]);

/* Number of host threads the parallel loops use (OpenMP's maximum; 1 without OpenMP). */
int lbm_oracle_threads(void);

/* Set the number of host threads for the parallel loops that follow (n >= 1; ignored
 * without OpenMP).  Used to time the oracle on one core. */
void lbm_oracle_set_threads(int n);

/* f = E(rho0, u_b0): post-streaming populations at t = 0.  uz0/ur0 may be NULL (0). */
int lbm_oracle_init(const lbm_oracle_params* p, const double* rho0, const double* uz0,
                    const double* ur0, double* f);

/* Advance the post-streaming populations f by nsteps time steps in place. */
int lbm_oracle_step(const lbm_oracle_params* p, double* f, int64_t nsteps);

/* Density and physical velocity u = (j + F/2)/rho of the state f. */
int lbm_oracle_moments(const lbm_oracle_params* p, const double* f, double* rho, double* uz,
                       double* ur);

/* sum over nodes of 2 pi r_j rho (axisymmetric mass). */
int lbm_oracle_mass(const lbm_oracle_params* p, const double* f, double* mass);

/* Mean P_k(rho) over nodes at distance < r_in from (zc, 0) minus the mean over
 * nodes at distance > r_out; distance measured in the (z, r) plane. */
int lbm_oracle_laplace(const lbm_oracle_params* p, const double* f, double zc, double r_in,
                       double r_out, double* dp);

/* Position of the drop's interface on the symmetry axis (Sec. 3.2): along row j = 0 from
 * column floor(zc) towards +z, the first k whose next node has rho <= thr, interpolated
 * linearly, z = k + (rho_k - thr) / (rho_k - rho_{k+1}); NaN if none before the last column. */
int lbm_oracle_axis_interface(const lbm_oracle_params* p, const double* f, double zc, double thr,
                              double* z);

#ifdef __cplusplus
}
#endif
#endif
