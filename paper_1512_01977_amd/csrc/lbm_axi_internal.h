// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbm_axi.h"

namespace lbm {

lbm_status eos_critical(const lbm_axi_params& p, double* rho_c, double* T_c, double* P_c);
lbm_status eos_coexistence(const lbm_axi_params& p, double* rho_v, double* rho_l, double* p_sat);
double eos_psi(const lbm_axi_params& p, double rho);  // sqrt(rho/3 - P_k), 0 for the ideal gas

// Per-instance constants as the kernels read them (uniform, loaded through the scalar cache).
struct InstDev {
  long long base;    // element index of the instance's first row block in a distribution buffer
  int nz, nr;
  int pitch;         // elements of one row of one plane (nz rounded up to 128 bytes); a row
                     // block holds the nine planes' rows: element (i, row, col) at
                     // base + (9 row + i) pitch + col
  int eos, axisym, faxis_sound, bc_top, forcing, source_mid;
  // EOS in the form the kernels evaluate (FP64 in every precision):
  //   Carnahan-Starling  P = c1 rho n(e) / (1 - e)^3 - c2 rho^2, e = ce rho (c1 = lambda R T, c2 = lambda a, ce = b / 4)
  //   van der Waals      P = c1 rho / (3 - rho) - c2 rho^2       (c1 = 8 lambda T, c2 = 3 lambda)
  // rmax: the density where the repulsive term diverges (the EOS domain ends there).
  double c1, c2, ce, rmax;
  double A, omega, nu, gz; // A, 1/tau, (tau - 1/2)/3, body force density
  // Storage shift: the planes hold g_i = f_i - w_i rho_ref and the psi ring holds
  // psi - psi_ref, psi_ref = psi(rho_ref).  In FP32 this keeps the momentum (a small
  // difference of O(rho) populations) and the psi gradients at full relative precision;
  // FP64 uses rho_ref = psi_ref = 0.
  double rho_ref, psi_ref, psi_ref2;  // psi_ref2 = psi_ref^2
};

// One unit of work of the fused step kernel: a strip of output columns
// [k0, k0 + ncols) of instance `inst`, rows [s, e).
struct WorkItem {
  int inst, k0, ncols, s, e;
};

// Rows of the distribution planes start on 128-byte boundaries and the step kernel's strips
// of output columns are whole 128-byte lines, so that no line is written in part by two
// workgroups (HBM has no byte masks: a partly written line costs a read-modify-write).
// The nine planes of a row sit next to each other (a row block), so that the rows a
// workgroup reads and writes in one step are close together in memory.
inline int line_elems(int esize) { return 128 / esize; }
// A pitch that is a multiple of 2 KiB gets one more line, so that the nine planes of a row
// block do not sit at a power-of-two stride (measured 1-1.5 % faster on 16384-wide rows).
inline int row_pitch(int nz, int esize) {
  const int p = (nz + line_elems(esize) - 1) / line_elems(esize) * line_elems(esize);
  return (p * esize) % 2048 == 0 ? p + line_elems(esize) : p;
}
inline int strip_cols(int width, int esize) {
  // output columns of a workgroup of `width` lanes: six halo lanes on either side (seven
  // with the link-midpoint source; for every width and element size the whole lines that
  // fit are the same either way)
  return (width - 14) / line_elems(esize) * line_elems(esize);
}

// Rows of one work item of the step kernel (its segment plus up to 16 rows of pipeline and
// gather halo: 7 on either side with the link-midpoint source, and the gather's row beyond)
// stay within 2 GiB of its load descriptor's base: the segment length cap.
inline int max_item_rows(int pitch, int esize) {
  const long long block = 9LL * pitch * esize;
  const long long rows = (1LL << 31) / block - 16;
  return rows > (1 << 30) ? (1 << 30) : (int)rows;
}

// Arguments of the fused step kernel.
template <typename R>
struct SweepArgs {
  const R* __restrict__ fin;   // post-collision planes of the previous step
  R* __restrict__ fout;        // post-collision planes of this step
  const InstDev* __restrict__ inst;
  const WorkItem* __restrict__ items;
  int n_items;
  int xcd_swizzle;
  int* queue;                  // [0] next ticket, [1] finished workgroups (persistent launches)
  int* err;                    // sticky device error bits: [0] any instance, [1 + k] instance k
  double* mrho;                // moments outputs (moments launches only), instance-local [nr][nz]
  double* muz;
  double* mur;
};

struct RowRef {
  int inst, row;
};

template <typename R>
hipError_t sweep_dispatch(const SweepArgs<R>& g, int width, bool moments, bool persist, bool regf, bool guo,
                          bool mid, int grid, hipStream_t st);
template <typename R>
hipError_t launch_unstream(R* fout, int nz, int pitch, int nr, int bc_top, double rho_ref,
                           const double* rho0,
                           const double* uz0, const double* ur0, const double* f0, hipStream_t st);
template <typename R>
hipError_t launch_export(const R* fin, int nz, int pitch, int nr, int bc_top, double rho_ref,
                         double* out, hipStream_t st);
template <typename R>
hipError_t launch_rows(int K, const R* fin, const InstDev* inst, const RowRef* rows,
                       int nrows, const double* geo, double* part, hipStream_t st);
template <typename R>
hipError_t launch_axis(const R* fin, const InstDev* inst, int n, const double* geo, double* out, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, long long bytes, hipStream_t st);
hipError_t launch_finish(int K, const double* part, const int* row_start, const InstDev* inst, int n,
                         double* out, hipStream_t st);

}  // namespace lbm
