/*
 * lbm_axi.h -- C ABI of the MI355X axisymmetric multiphase lattice Boltzmann library.
 *
 * The library advances the D2Q9 BGK lattice Boltzmann method on the (z, r)
 * half-plane of Reijers, Gelderblom and Toschi (arXiv:1512.01977):
 *   - pull streaming with mid-grid specular reflection at the axis r = 0 and a
 *     free-slip (specular) or no-slip (half-way bounce-back) wall at r = nr,
 *     periodic in z (Sec. 3.1-3.3);
 *   - density and momentum moments, physical velocity u = (j + F/2)/rho (Sec. 2.1);
 *   - a generic equation of state P_k(rho) and the pseudopotential
 *     psi = sqrt(rho/3 - P_k) (Sec. 2.3);
 *   - the Kupershtokh single-neighbour force, eq. (kupershtokhforcing), applied
 *     with the exact-difference method (Sec. 2.3);
 *   - the axisymmetric force correction F_axis, eq. (multiphasecorrections), with
 *     the isotropic stencils of eq. (fifthorderaccuratefinitedifference);
 *   - the axisymmetric source h_i of eq. (axihz) (Sec. 2.2) and BGK collision,
 *     eq. (lbm).
 * All of that runs in HIP kernels for gfx950; the host side only validates
 * arguments, lays out memory and launches.
 *
 * Grid: node (k, j) sits at z = k (k = 0..nz-1) and r = j + 1/2 (j = 0..nr-1).
 * Host node fields are double arrays [nr][nz] (k fastest); a distribution is
 * double [9][nr][nz] in the direction order
 *   0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
 * with components (c_z, c_r).
 *
 * Conventions for every entry point:
 *   - returns LBM_OK (0) or a negative lbm_status; nothing throws across the ABI;
 *   - host arrays are owned by the caller and only read or written during the call;
 *   - device memory is owned by the library unless a workspace is adopted
 *     (lbm_axi_batch_init_ws), in which case the caller keeps it alive until
 *     lbm_axi_destroy and the library never frees it;
 *   - a handle is bound to one HIP stream and is not thread-safe;
 *   - lbm_axi_step is asynchronous; errors raised on the device (EOS domain,
 *     non-finite values) are reported by the next synchronising call: lbm_axi_sync,
 *     _mass and _laplace report them for any instance, _moments and _get_f for the
 *     instance they read (instances are independent).
 */
#ifndef LBM_AXI_H
#define LBM_AXI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
#define LBM_OK 0
#define LBM_ERR_ARG (-1)         /* invalid argument or parameter set */
#define LBM_ERR_ALLOC (-2)       /* device or host allocation failed, or workspace too small */
#define LBM_ERR_HIP (-3)         /* a HIP runtime call failed */
#define LBM_ERR_EOS_DOMAIN (-4)  /* rho <= 0 or rho/3 - P_k < 0 (psi not real) on some node */
#define LBM_ERR_NONFINITE (-5)   /* a non-finite value appeared */
#define LBM_ERR_UNSUPPORTED (-6) /* valid request outside what the library supports (see calls) */

typedef enum { LBM_EOS_IDEAL = 0, LBM_EOS_VDW = 1, LBM_EOS_CS = 2 } lbm_eos_kind;
typedef enum { LBM_TOP_FREE_SLIP = 0, LBM_TOP_NO_SLIP = 1 } lbm_top_bc;
typedef enum { LBM_PREC_FP64 = 0, LBM_PREC_FP32 = 1 } lbm_precision;
typedef enum { LBM_FORCING_EDM = 0, LBM_FORCING_GUO = 1 } lbm_forcing;

/* One simulation instance.  Sec. 2 of the paper defines every field except
 * the Carnahan-Starling coefficients, which follow the usual form
 *   P = lambda [rho R T (1 + e + e^2 - e^3)/(1 - e)^3 - a rho^2],  e = b rho / 4. */
typedef struct {
  int32_t nz, nr;            /* nz >= 1, nr >= 4 */
  double tau;                /* BGK relaxation time > 1/2; nu = (tau - 1/2)/3 */
  int32_t eos;               /* lbm_eos_kind */
  double T;                  /* absolute EOS temperature (vdW: T/T_c since that EOS is reduced) */
  double eos_a, eos_b, eos_R;/* Carnahan-Starling a, b, R (ignored otherwise) */
  double lambda;             /* pressure scale of eq. (kupershtokvdwpressure); also scales CS */
  double A;                  /* Kupershtokh mixing parameter, eq. (kupershtokhforcing) */
  int32_t axisym;            /* 1: h_i and F_axis on (axisymmetric); 0: plain 2-D (z, r) plane */
  int32_t faxis_sound;       /* 0: F_axis uses c_k^4 = (dP_k/drho)^2 (Sec. 2.3); 1: c_s^4 = 1/9 */
  int32_t bc_top;            /* lbm_top_bc at r = nr */
  double gz;                 /* uniform body-force density along z added to F */
  int32_t forcing;           /* lbm_forcing: LBM_FORCING_EDM, the exact-difference method the
                                paper relies on (Sec. 2.3, default), or LBM_FORCING_GUO, the
                                source term printed in Sec. 2.1 (its second term read as
                                (c_i.u)(c_i.F)/c_s^4, BGK toward E(rho, u), u = (j + F/2)/rho) */
  int32_t source_mid;        /* 0: the source h_i of eq. (axihz) from the fields at the node (x, t)
                                (default); 1: at the link midpoint x + c_i/2 where the evolution
                                equation of Sec. 2.2 places it, as the mean of h_i at x and at
                                x + c_i (both at time t; beyond the axis or the wall the mirror
                                node's source in the mirrored direction).  Launches holding such
                                an instance run a pipeline one row deeper.  Other values:
                                LBM_ERR_ARG */
} lbm_axi_params;

/* Launch shape of the fused step kernel (chosen by lbm_axi_autotune or set by hand). */
typedef struct {
  int32_t width;        /* lanes per workgroup along z: 64, 128 or 256; a workgroup writes the
                           whole 128-byte lines that fit in width - 12 columns (12 are halo) */
  int32_t seg_rows;     /* rows of r per work item (>= 8), 0 = whole column; capped so that
                           a work item's rows span less than 2 GiB (wide FP64 rows) */
  int32_t persistent;   /* 1: persistent grid draining a work queue; 0: one workgroup per item */
  int32_t grid;         /* persistent grid size, 0 = automatic */
  int32_t xcd_swizzle;  /* 1: neighbouring work items go to the same XCD; 0: items longest
                           first, dealt round-robin over the XCDs (better balance); 2: longest
                           first, the strips of one row band on one XCD (their shared edge
                           lines stay in its L2); other values: LBM_ERR_ARG.  Ignored by the
                           persistent grid, which always takes items longest first */
  int32_t regf;         /* 1: carry gathered populations in registers (no second gather; the
                           default except in FP64 with the link-midpoint source); 0: gather
                           them again for the collision.  Both give the same results */
  int32_t streams;      /* 1 (or 0): one launch per step for all instances; 2..4: the instances
                           of a batch split into this many groups of about equal node counts,
                           each stepped by its own launches on its own stream (created by the
                           library, default priority), forked from and joined back into the
                           handle's stream, so that one group's last work items overlap the
                           others' next step.  Needs streams <= number of instances, else
                           LBM_ERR_ARG.  Results do not depend on it. */
} lbm_axi_launch;

typedef struct lbm_axi_s* lbm_axi_t;

/* Human-readable name of a status code (static storage). */
const char* lbm_axi_status_string(lbm_status s);

/* ---------------------------------------------------------------- host helpers */

/* Critical point of the EOS in p (p->T ignored): dP/drho = d2P/drho2 = 0 (Sec. 2.3 for
 * vdW; CS in the same slot).  Outputs are host scalars.  LBM_ERR_ARG for NULL pointers,
 * the ideal gas (no critical point) or non-positive CS coefficients. */
lbm_status lbm_axi_eos_critical(const lbm_axi_params* p, double* rho_c, double* T_c, double* P_c);

/* Maxwell equal-area coexistence densities and saturation pressure at p->T < T_c (the
 * densities Sec. 2.3 compares the EDM coexistence curve with).  Outputs are host scalars.
 * LBM_ERR_ARG for NULL pointers, the ideal gas, or T >= T_c. */
lbm_status lbm_axi_eos_coexistence(const lbm_axi_params* p, double* rho_v, double* rho_l,
                                   double* p_sat);

/* ---------------------------------------------------------------- lifetime */

/* Single instance: allocate device state and set f = E(rho0, u0) (eq. lbm's
 * equilibrium, Sec. 2.1) as the populations after streaming at t = 0.
 * rho0: host [nr][nz], required; uz0, ur0: host [nr][nz] or NULL for 0.
 * precision: lbm_precision.  stream: hipStream_t, NULL = the library creates its own.
 * Errors: LBM_ERR_ARG (NULL out/rho0, nz < 1, nr < 4, nz*nr > 2^31, tau <= 1/2, unknown
 * eos/bc/forcing/flag, non-finite A, gz or T, CS b <= 0, lambda <= 0 for a non-ideal EOS);
 * LBM_ERR_NONFINITE / LBM_ERR_EOS_DOMAIN (rho0 non-finite, <= 0, or psi not real);
 * LBM_ERR_UNSUPPORTED (rows so wide that 22 of them, nine planes each, span 2 GiB or more,
 * about nz > 1.4e6 in FP64: the step kernel addresses the rows of a work item with 32-bit
 * offsets); LBM_ERR_ALLOC; LBM_ERR_HIP.  *out is NULL on error. */
lbm_status lbm_axi_init(const lbm_axi_params* p, int32_t precision, const double* rho0,
                        const double* uz0, const double* ur0, void* stream, lbm_axi_t* out);

/* n independent instances (uneven sizes and parameters) advanced together by one
 * launch per step.  params[k] and rho0[k] (host [nr_k][nz_k]) describe instance k.
 * Errors as lbm_axi_init, for any instance (n < 1: LBM_ERR_ARG). */
lbm_status lbm_axi_batch_init(int32_t n, const lbm_axi_params* params, int32_t precision,
                              const double* const* rho0, void* stream, lbm_axi_t* out);

/* Device bytes needed for the two distribution buffers of an n-instance batch (host
 * arithmetic only).  Errors: LBM_ERR_ARG (as lbm_axi_batch_init's parameter checks),
 * LBM_ERR_UNSUPPORTED (rows too wide for the step kernel's 32-bit offsets, as for
 * lbm_axi_init; nothing to allocate). */
lbm_status lbm_axi_workspace_bytes(int32_t n, const lbm_axi_params* params, int32_t precision,
                                   size_t* bytes);

/* As lbm_axi_batch_init, but the distribution buffers live in a caller-owned
 * device workspace of at least lbm_axi_workspace_bytes bytes (256-byte aligned).  The
 * caller keeps it alive until lbm_axi_destroy.  LBM_ERR_ALLOC if it is too small. */
lbm_status lbm_axi_batch_init_ws(int32_t n, const lbm_axi_params* params, int32_t precision,
                                 const double* const* rho0, void* stream, void* workspace,
                                 size_t workspace_bytes, lbm_axi_t* out);

/* Release everything the library allocated; NULL is a no-op. */
void lbm_axi_destroy(lbm_axi_t h);

/* ---------------------------------------------------------------- time stepping */

/* Enqueue nsteps >= 0 time steps of every instance on the handle's stream (Sec. 2:
 * streaming, moments, EOS and psi, F_K + F_axis, h_i, exact-difference BGK).  With a
 * launch shape of several stream groups the steps run on the groups' streams, after the
 * work already on the handle's stream and before any work enqueued on it later.  Returns
 * before the steps run; LBM_ERR_ARG for a NULL handle or nsteps < 0, LBM_ERR_HIP if a
 * launch or a graph capture fails.  Device-side errors surface at the next synchronising
 * call. */
lbm_status lbm_axi_step(lbm_axi_t h, int64_t nsteps);

/* As lbm_axi_step, then wait; *ms receives the HIP-event time of the launches
 * on the handle's stream (kernel time, no host overhead between steps; with stream
 * groups, from before the first group's first launch to after the last group's last). */
lbm_status lbm_axi_step_timed(lbm_axi_t h, int64_t nsteps, double* ms);

/* Wait for the stream and report any device-side error. */
lbm_status lbm_axi_sync(lbm_axi_t h);

/* Per-instance device error bits (1: EOS domain left, 2: non-finite value; 0 = clean),
 * flags is host int32 [n].  Synchronises; the bits stay set (the state is invalid). */
lbm_status lbm_axi_errors(lbm_axi_t h, int32_t* flags);

/* Replay steps as captured hipGraphs of `chunk` steps (even, >= 2); 0 = eager launches.
 * The chunks starting from either buffer are captured and uploaded by this call (no step
 * runs; the call waits for the uploads), so that no step call spends host time capturing.
 * A later set_launch drops them (captured again when a step next needs one).  LBM_ERR_ARG
 * for an odd or negative chunk, LBM_ERR_HIP if the capture fails. */
lbm_status lbm_axi_set_graph_chunk(lbm_axi_t h, int32_t chunk);

/* ---------------------------------------------------------------- observables (synchronising) */

/* rho and the physical velocity u = (j + F/2)/rho (Sec. 2.1) of instance k; host [nr][nz]
 * outputs (caller-owned).  LBM_ERR_ARG for a bad k or NULL output; LBM_ERR_EOS_DOMAIN or
 * LBM_ERR_NONFINITE if instance k has left the EOS domain (the outputs are then filled but
 * meaningless).  The first call allocates a device buffer for three fields of the largest
 * instance and the per-instance work lists, kept until lbm_axi_destroy (rebuilt after a
 * change of strip width or segment length). */
lbm_status lbm_axi_moments(lbm_axi_t h, int32_t k, double* rho, double* uz, double* ur);

/* mass[k] = sum over nodes of 2 pi r_j rho, FP64, deterministic; mass is host [n]. */
lbm_status lbm_axi_mass(lbm_axi_t h, double* mass);

/* For callers that cannot allocate device memory or synchronise (code under stream capture,
 * tight serving loops): lbm_axi_mass without allocation or host round trip.  Enqueues on the
 * handle's stream the same fixed-order FP64 reduction, whose per-row partials live in the
 * library's static device scratch (1 MiB per GPU, held until the process ends: at most
 * 131072 rows over all instances of the handle, else LBM_ERR_UNSUPPORTED), and writes the n
 * per-instance masses to mass_dev, a caller-owned device array of n doubles on the handle's
 * device.  The result equals lbm_axi_mass's bitwise once the stream has reached it.  Allocates
 * nothing and does not synchronise; device errors of the state are not reported here (call
 * lbm_axi_sync).  Every call on one GPU shares that GPU's scratch: calls that overlap in time
 * on one GPU (handles on different streams) race and must be ordered by the caller. */
lbm_status lbm_axi_mass_async(lbm_axi_t h, double* mass_dev);

/* dp[k] = mean P_k(rho) over nodes closer than r_in[k] to (zc[k], 0) minus the mean
 * over nodes farther than r_out[k] (Young-Laplace, eq. laplacepressure); host [n] arrays. */
lbm_status lbm_axi_laplace(lbm_axi_t h, const double* zc, const double* r_in,
                           const double* r_out, double* dp);

/* Where each drop's interface crosses the symmetry axis, the observable Sec. 3.2 follows
 * for the oscillating drop: on the axis row (j = 0), from column floor(zc[k]) towards +z,
 * the first column k whose next node has rho <= thr[k], and z[k] = k + (rho_k - thr) /
 * (rho_k - rho_{k+1}) (linear interpolation; NaN when no column before the last
 * qualifies).  zc, thr, z: host [n] arrays.  Errors: LBM_ERR_ARG (zc outside [0, nz) or
 * a non-finite thr); device errors as lbm_axi_sync.  Synchronising. */
lbm_status lbm_axi_axis_interface(lbm_axi_t h, const double* zc, const double* thr, double* z);

/* Checkpoint: the post-streaming populations of instance k as host double [9][nr][nz]. */
lbm_status lbm_axi_get_f(lbm_axi_t h, int32_t k, double* f);

/* Resume: replace the state of instance k by host double [9][nr][nz] post-streaming populations. */
lbm_status lbm_axi_set_f(lbm_axi_t h, int32_t k, const double* f);

/* ---------------------------------------------------------------- launch shape and tuning */

lbm_status lbm_axi_get_launch(lbm_axi_t h, lbm_axi_launch* cfg);
lbm_status lbm_axi_set_launch(lbm_axi_t h, const lbm_axi_launch* cfg);

/* Time every candidate launch shape for steps_per_trial steps (state saved and
 * restored on the device), keep the fastest, return it and its ms per step.  A handle
 * whose state has already raised a sticky device error is not tuned: the call returns
 * that error (LBM_ERR_EOS_DOMAIN / LBM_ERR_NONFINITE) and leaves the error words, the
 * state and the launch shape as they were.  Synchronising; allocates a copy of one
 * distribution buffer for the duration of the call. */
lbm_status lbm_axi_autotune(lbm_axi_t h, int32_t steps_per_trial, lbm_axi_launch* best,
                            double* best_ms_per_step);

/* Measurement reference, not part of the method: copy `bytes` (a multiple of 16) between
 * two device buffers the call allocates, `iters` times on the null stream, and return the
 * read+write rate in GB/s.  Gives the practical HBM copy ceiling and a kernel of known
 * traffic for calibrating profiler byte counters.  Synchronising. */
lbm_status lbm_axi_stream_copy(int64_t bytes, int32_t iters, double* gbps);

/* Sizes: number of instances, total nodes, and bytes of one distribution buffer. */
lbm_status lbm_axi_sizes(lbm_axi_t h, int32_t* n, int64_t* nodes, int64_t* f_bytes);

#ifdef __cplusplus
}
#endif
#endif
