// HIP kernels of the axisymmetric multiphase lattice Boltzmann step (arXiv:1512.01977)
// for gfx950.  See lbm_axi.h for conventions.
//
// Fused step kernel ("sweep").  One workgroup of W lanes owns a strip of output
// columns (z, contiguous in memory; whole 128-byte lines, at most W - 12 columns)
// plus a 6-column halo on each side, and walks up the rows (r) of one segment.
// Every iteration t advances four pipeline stages that lag each other by two rows:
//   A (row t)    pull-gather the 9 populations with the wall maps, moments rho and
//                j, EOS in FP64: P_k, kappa = dP_k/drho, psi = sqrt(rho/3 - P_k)
//   B (row t-2)  D_z psi, D_r psi (eq. fifthorderaccuratefinitedifference) and
//                the Kupershtokh force F_K (eq. kupershtokhforcing)
//   C (row t-4)  D_rr psi = D_r(D_r psi), D_rz psi = D_r(D_z psi), F_axis
//                (eq. multiphasecorrections), F, physical velocity u = (j + F/2)/rho
//   D (row t-6)  D_r u_z, D_z u_r, D_r u_r, H and h_i (eq. axihz), the forcing
//                (exact difference, or Guo's term per instance) + BGK (eq. lbm),
//                store the post-collision populations
// Each stage's stencil input lives in a 5-row LDS ring (psi, D_z psi, D_r psi,
// u_z, u_r); values a stage needs only at its own node travel in registers.
// Ghost rows across the axis and the outer wall are written into the rings by the
// producing stage with the field's mirror parity, so the stencils never branch.
// Nothing but the populations touches HBM: one read and one write per node, in row
// blocks (the nine planes' rows of one r side by side).  The workgroup barriers order
// LDS only, and each row is gathered one iteration before it is used, so the loads and
// stores stay in flight across the pipeline steps.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lbm_axi_internal.h"

namespace lbm {

constexpr int RD = 5;  // ring depth: a radius-2 stencil reads 5 consecutive rows
enum { R_PSI = 0, R_DZ = 1, R_DR = 2, R_UZ = 3, R_UR = 4, NRING = 5, R_FKZ = 5, R_FKR = 6 };
// Fields of the LDS rings: five, and two more (F_K) in FP64 with the populations in registers
// (run_item's LEAN form).
template <typename R, bool MOMENTS, bool REGF, bool MID>
constexpr int ring_fields() {
  return REGF && sizeof(R) == 8 && !MID && !MOMENTS ? 7 : NRING;
}
enum { ERR_BIT_DOMAIN = 1, ERR_BIT_NONFINITE = 2 };

__device__ __forceinline__ int wrapi(int x, int n) {
  int r = x % n;
  return r < 0 ? r + n : r;
}
__device__ __forceinline__ int slot(int x) {
  int r = x % RD;
  return r < 0 ? r + RD : r;
}

// Workgroup barrier that orders LDS only.  The stages exchange data through LDS alone, so
// the barrier need not wait for the wave's outstanding global loads and stores (a full
// __syncthreads() does, which would expose the HBM latency at every pipeline step).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Reciprocals: hardware estimate refined by Newton steps (one for FP32, two for FP64),
// within an ulp of 1/x; used instead of IEEE division on the hot path.
__device__ __forceinline__ float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  const float e = __builtin_fmaf(-x, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Fused multiply-add in the storage precision (the plain builtin would promote floats).
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// P_k and kappa = dP_k/drho in FP64 (Sec. 2.3; Carnahan-Starling in the same slot), from the
// per-instance constants c1, c2, ce (see InstDev).
__device__ __forceinline__ void eos_dev(const InstDev& I, double rho, double& P, double& kap) {
  if (I.eos == LBM_EOS_CS) {
    const double e = I.ce * rho;
    const double im = recip(1.0 - e);
    const double im3 = im * im * im;
    const double num = 1.0 + e * (1.0 + e * (1.0 - e));
    const double dnum = 1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)));
    const double c2r = I.c2 * rho;
    P = __builtin_fma(I.c1 * rho * num, im3, -c2r * rho);
    kap = __builtin_fma(I.c1 * dnum, im3 * im, -2.0 * c2r);
  } else if (I.eos == LBM_EOS_VDW) {
    const double id = recip(3.0 - rho);
    const double c2r = I.c2 * rho;
    P = __builtin_fma(I.c1 * rho, id, -c2r * rho);
    kap = __builtin_fma(3.0 * I.c1 * id, id, -2.0 * c2r);
  } else {
    P = rho * (1.0 / 3.0);
    kap = 1.0 / 3.0;
  }
}

// Post-streaming populations of node (col, x) pulled from the post-collision
// populations f of one instance: f_i(x) = f*_i(x - c_i), with mid-grid specular reflection
// at the axis, specular (free slip) or half-way bounce-back (no slip) at r = nr, periodic z.
// cm, c0, cp are the wrapped columns k-1, k, k+1.  Layout: row blocks of the nine direction
// planes, element (i, row, col) at (9 row + i) pitch + col.
template <typename R>
__device__ __forceinline__ void gather(const R* __restrict__ f, int pitch, int nr, int bc_top,
                                       int x, unsigned cm, unsigned c0, unsigned cp, R o[9]) {
  const long long P = pitch, rs = 9LL * pitch;
  const R* r0 = f + (long long)x * rs;
  const R* rm = x > 0 ? r0 - rs : r0;       // row x-1 feeds the directions with c_r = +1
  const R* rp = x < nr - 1 ? r0 + rs : r0;  // row x+1 feeds the directions with c_r = -1
  o[0] = r0[c0];
  o[1] = (r0 + P)[cm];
  o[3] = (r0 + 3 * P)[cp];
  if (x > 0) {
    o[2] = (rm + 2 * P)[c0];
    o[5] = (rm + 5 * P)[cm];
    o[6] = (rm + 6 * P)[cp];
  } else {  // axis: (c_z, +1) arrives from (c_z, -1) leaving node (k - c_z, 0)
    o[2] = (r0 + 4 * P)[c0];
    o[5] = (r0 + 8 * P)[cm];
    o[6] = (r0 + 7 * P)[cp];
  }
  if (x < nr - 1) {
    o[4] = (rp + 4 * P)[c0];
    o[7] = (rp + 7 * P)[cp];
    o[8] = (rp + 8 * P)[cm];
  } else if (bc_top == LBM_TOP_FREE_SLIP) {  // (c_z, -1) from (c_z, +1) at (k - c_z, nr-1)
    o[4] = (r0 + 2 * P)[c0];
    o[7] = (r0 + 6 * P)[cp];
    o[8] = (r0 + 5 * P)[cm];
  } else {  // bounce-back: (-c_z, -1) from (c_z, +1) of the same node
    o[4] = (r0 + 2 * P)[c0];
    o[7] = (r0 + 5 * P)[c0];
    o[8] = (r0 + 6 * P)[c0];
  }
}

// The same pull map through raw buffer loads: one 128-bit descriptor based at the first
// row block a work item touches, with the row and the plane as a uniform byte offset and
// the column as a per-lane byte offset, so that no per-lane address arithmetic is spent on
// the loads.  The host keeps the rows of a work item within 2 GiB of that base.
template <typename R>
struct Planes {
  __amdgpu_buffer_rsrc_t g;
  unsigned pstride;  // bytes between consecutive planes of a row block
  unsigned rstride;  // bytes between consecutive row blocks
};

// nbytes: the descriptor's range; a raw-buffer access at an offset past it is dropped by
// the hardware (a store writes nothing, a load returns 0).
template <typename R>
__device__ __forceinline__ Planes<R> make_planes(const R* base, int pitch, unsigned nbytes = 0xffffffffu) {
  Planes<R> p;
  p.g = __builtin_amdgcn_make_buffer_rsrc(const_cast<R*>(base), (short)0, (int)nbytes, (int)0x00020000);
  p.pstride = (unsigned)pitch * (unsigned)sizeof(R);
  p.rstride = 9u * p.pstride;
  return p;
}

__device__ __forceinline__ float bload(float, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ double bload(double, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 0);
}


// bm, b0, bp: byte offsets of columns k-1, k, k+1 within a row; x0: the row the
// descriptor is based at.  The wall cases are chosen with uniform selects of the plane
// and row offsets (and, at a no-slip wall, of the column), so that the nine loads form one
// straight sequence: the compiler can then track them individually and overlap them with
// the stores still in flight.
template <typename R>
__device__ __forceinline__ void gather_b(const Planes<R>& pl, int nr, int bc_top, int x, int x0, unsigned bm,
                                         unsigned b0, unsigned bp, R o[9]) {
  const unsigned rs = pl.rstride, ps = pl.pstride;
  const unsigned s0 = (unsigned)(x - x0) * rs;
  const bool axis = x == 0, top = x == nr - 1;
  const bool noslip = top && bc_top == LBM_TOP_NO_SLIP;
  const unsigned sm = s0 - rs, sp = s0 + rs;
  o[0] = bload(R(0), pl.g, b0, s0);
  o[1] = bload(R(0), pl.g, bm, s0 + ps);
  o[3] = bload(R(0), pl.g, bp, s0 + 3 * ps);
  // c_r = +1 from row x - 1; across the axis (c_z, +1) is (c_z, -1) of node (k - c_z, 0)
  o[2] = bload(R(0), pl.g, b0, axis ? s0 + 4 * ps : sm + 2 * ps);   // 4 : 2
  o[5] = bload(R(0), pl.g, bm, axis ? s0 + 8 * ps : sm + 5 * ps);   // 8 : 5
  o[6] = bload(R(0), pl.g, bp, axis ? s0 + 7 * ps : sm + 6 * ps);   // 7 : 6
  // c_r = -1 from row x + 1; at the wall from (c_z, +1) of node (k - c_z, nr - 1)
  // (specular) or of the same node with c_z reversed (bounce-back)
  o[4] = bload(R(0), pl.g, b0, top ? s0 + 2 * ps : sp + 4 * ps);    // 2 : 4
  o[7] = bload(R(0), pl.g, noslip ? b0 : bp, top ? (noslip ? s0 + 5 * ps : s0 + 6 * ps) : sp + 7 * ps);  // 5 | 6 : 7
  o[8] = bload(R(0), pl.g, noslip ? b0 : bm, top ? (noslip ? s0 + 6 * ps : s0 + 5 * ps) : sp + 8 * ps);  // 6 | 5 : 8
}

// gather_b for an interior row (0 < x < nr - 1): the same loads in the same order, without
// the wall selects; gather_row() picks it for interior rows (a uniform branch).
template <typename R>
__device__ __forceinline__ void gather_interior(const Planes<R>& pl, int x, int x0, unsigned bm, unsigned b0,
                                                unsigned bp, R o[9]) {
  const unsigned rs = pl.rstride, ps = pl.pstride;
  const unsigned s0 = (unsigned)(x - x0) * rs, sm = s0 - rs, sp = s0 + rs;
  o[0] = bload(R(0), pl.g, b0, s0);
  o[1] = bload(R(0), pl.g, bm, s0 + ps);
  o[3] = bload(R(0), pl.g, bp, s0 + 3 * ps);
  o[2] = bload(R(0), pl.g, b0, sm + 2 * ps);
  o[5] = bload(R(0), pl.g, bm, sm + 5 * ps);
  o[6] = bload(R(0), pl.g, bp, sm + 6 * ps);
  o[4] = bload(R(0), pl.g, b0, sp + 4 * ps);
  o[7] = bload(R(0), pl.g, bp, sp + 7 * ps);
  o[8] = bload(R(0), pl.g, bm, sp + 8 * ps);
}

template <typename R>
__device__ __forceinline__ void gather_row(const Planes<R>& pl, int nr, int bc_top, int x, int x0, unsigned bm,
                                           unsigned b0, unsigned bp, R o[9]) {
  if (x > 0 && x < nr - 1)
    gather_interior<R>(pl, x, x0, bm, b0, bp, o);
  else
    gather_b<R>(pl, nr, bc_top, x, x0, bm, b0, bp, o);
}

// Equilibrium of Sec. 2.1 (c_s^2 = 1/3) relative to the storage shift:
// E_i(rho, u) - w_i rho_ref = w_i [(rho - rho_ref) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)],
// with sg = rho - rho_ref as summed from the shifted populations.
template <typename R>
__device__ __forceinline__ void shifted_equilibrium(R rho, R sg, R uz, R ur, R e[9]) {
  const R w0 = R(4.0 / 9.0), w1 = R(1.0 / 9.0), w2 = R(1.0 / 36.0);
  const R m = R(-1.5) * (uz * uz + ur * ur);
  auto E = [&](R w, R cu) { return w * (sg + rho * (m + R(3.0) * cu + R(4.5) * cu * cu)); };
  e[0] = w0 * (sg + rho * m);
  e[1] = E(w1, uz);
  e[2] = E(w1, ur);
  e[3] = E(w1, -uz);
  e[4] = E(w1, -ur);
  e[5] = E(w2, uz + ur);
  e[6] = E(w2, -uz + ur);
  e[7] = E(w2, -uz - ur);
  e[8] = E(w2, uz - ur);
}

// LDS rings, interleaved: element (ring q, row slot s, column c) sits at
// [s][c][q], so the five fields of one column are adjacent and a whole row of
// stencil reads (columns lane .. lane + 4) lies within 100 bytes of one base.  Every
// access is one per-lane base plus the uniform slot offset (rb = s * ROWB) plus an
// immediate; lanes step NF elements apart (NF = 5: an odd dword stride in FP32, no bank
// conflicts).
template <typename R, int W, int NF = NRING>
struct Rings {
  static constexpr int ROWB = (W + 4) * NF * (int)sizeof(R);
  char* base;  // the ring array; rows are addressed by per-lane byte offsets (lane part included)
  __device__ __forceinline__ R& at(int q, int vb, int dz) const {
    return *reinterpret_cast<R*>(base + vb + ((2 + dz) * NF + q) * (int)sizeof(R));
  }
};

// A ring's five rows x-2 .. x+2 as per-lane byte offsets.
struct Rows5 {
  int m2, m1, s0, p1, p2;
};

// D_z g (eq. fifthorderaccuratefinitedifference): directions 1, 3, 5, 6, 7, 8, each
// 8 g(x + c_i) - g(x + 2 c_i) weighted by c_iz; unscaled (the caller multiplies by 1/36).
template <typename R, int W, int NF>
__device__ __forceinline__ R stencil_dz36(const Rings<R, W, NF>& L, int q, const Rows5& r) {
  const R a = (L.at(q, r.s0, 1) - L.at(q, r.s0, -1)) + (L.at(q, r.p1, 1) - L.at(q, r.p1, -1)) +
              (L.at(q, r.m1, 1) - L.at(q, r.m1, -1));
  const R b = (L.at(q, r.s0, 2) - L.at(q, r.s0, -2)) + (L.at(q, r.p2, 2) - L.at(q, r.p2, -2)) +
              (L.at(q, r.m2, 2) - L.at(q, r.m2, -2));
  return fmad(R(8), a, -b);
}

// D_r g: directions 2, 4, 5, 6, 7, 8 weighted by c_ir; unscaled.
template <typename R, int W, int NF>
__device__ __forceinline__ R stencil_dr36(const Rings<R, W, NF>& L, int q, const Rows5& r) {
  const R a = (L.at(q, r.p1, -1) + L.at(q, r.p1, 0) + L.at(q, r.p1, 1)) -
              (L.at(q, r.m1, -1) + L.at(q, r.m1, 0) + L.at(q, r.m1, 1));
  const R b = (L.at(q, r.p2, -2) + L.at(q, r.p2, 0) + L.at(q, r.p2, 2)) -
              (L.at(q, r.m2, -2) + L.at(q, r.m2, 0) + L.at(q, r.m2, 2));
  return fmad(R(8), a, -b);
}

// Post-collision populations of one node (eq. lbm with the force of eq. kupershtokhforcing
// and the source h_i of eq. axihz), in shifted storage g_i = f_i - w_i rho_ref,
// s = rho - rho_ref.  With E_i(rho, v) = w_i rho (1 + Q_i(v)),
// Q_i(v) = 3 c_i.v + 4.5 (c_i.v)^2 - 1.5 v.v, and h_i = w_i (m0 + 3 c_i.H), both force
// applications give  g*_i = (1 - omega) g_i + w_i [M + c_i.A.c_i + c_i.V]  exactly:
//  exact-difference method (Sec. 2.3), u_b = j/rho, u_a = u_b + F/rho:
//   f*_i = f_i + omega (E_i(rho, u_b) - f_i) + E_i(rho, u_a) - E_i(rho, u_b) + h_i,
//   A = 4.5 rho T, T = (omega - 1) u_b u_b + u_a u_a, M = omega s + m0 - 1.5 rho tr T,
//   V = 3 rho (omega u_b + F/rho) + 3 H;
//  Guo (Sec. 2.1), u = (j + F/2)/rho, p = 1 - omega/2:
//   f*_i = f_i + omega (E_i(rho, u) - f_i) + w_i p [3 (c_i - u).F + 9 (c_i.u)(c_i.F)] + h_i,
//   A = 4.5 omega rho u u + 4.5 p (u F + F u), M = omega s + m0 - 1.5 omega rho u.u - 3 p u.F,
//   V = 3 (omega rho u + p F) + 3 H.
// The bracket is assembled from M, Kz = M + A_zz, Kr = M + A_rr, Kd = M + A_zz + A_rr and
// X = 2 A_zr.  H3 = 3 H; F = (Fz, Fr).
template <typename R>
__device__ __forceinline__ void collide(const R g[9], R rho, R sg, R jz, R jr, R Fz, R Fr, R m0, R H3z, R H3r,
                                        R omega, bool guo, R out[9]) {
  const R w0 = R(4.0 / 9.0), w1 = R(1.0 / 9.0), w2 = R(1.0 / 36.0);
  const R irho = recip(rho);
  R M, Kz, Kr, Kd, X, Vz, Vr;
  if (!guo) {
    const R ubz = jz * irho, ubr = jr * irho;
    const R duz = Fz * irho, dur = Fr * irho;
    const R uaz = ubz + duz, uar = ubr + dur;
    const R om1 = omega - R(1);
    const R tz = om1 * ubz, tr = om1 * ubr;
    const R Tzz = fmad(tz, ubz, uaz * uaz);
    const R Trr = fmad(tr, ubr, uar * uar);
    const R Tzr = fmad(tz, ubr, uaz * uar);
    const R tT = Tzz + Trr;
    M = fmad(R(-1.5) * rho, tT, fmad(omega, sg, m0));
    const R r45 = R(4.5) * rho;
    Kz = fmad(r45, Tzz, M);
    Kr = fmad(r45, Trr, M);
    Kd = fmad(r45, tT, M);
    X = R(9) * rho * Tzr;
    const R r3 = R(3) * rho;
    Vz = fmad(r3, fmad(omega, ubz, duz), H3z);  // (omega - 1) u_b + u_a = omega u_b + du
    Vr = fmad(r3, fmad(omega, ubr, dur), H3r);
  } else {
    const R uz = fmad(R(0.5), Fz, jz) * irho, ur = fmad(R(0.5), Fr, jr) * irho;
    const R orho = omega * rho, p = R(1) - R(0.5) * omega;
    const R o45 = R(4.5) * orho, p9 = R(9) * p;
    const R uF = fmad(uz, Fz, ur * Fr);
    M = fmad(R(-1.5) * orho, fmad(uz, uz, ur * ur), fmad(omega, sg, m0)) - R(3) * p * uF;
    const R Azz = fmad(o45 * uz, uz, p9 * uz * Fz);
    const R Arr = fmad(o45 * ur, ur, p9 * ur * Fr);
    X = fmad(R(2) * o45 * uz, ur, p9 * fmad(uz, Fr, ur * Fz));
    Kz = M + Azz;
    Kr = M + Arr;
    Kd = Kz + Arr;
    Vz = fmad(R(3), fmad(orho, uz, p * Fz), H3z);
    Vr = fmad(R(3), fmad(orho, ur, p * Fr), H3r);
  }
  const R Kdp = Kd + X, Kdm = Kd - X;
  const R Sp = Vz + Vr, Sm = Vr - Vz;
  const R omc = R(1) - omega;
  out[0] = fmad(omc, g[0], w0 * M);
  out[1] = fmad(omc, g[1], w1 * (Kz + Vz));
  out[2] = fmad(omc, g[2], w1 * (Kr + Vr));
  out[3] = fmad(omc, g[3], w1 * (Kz - Vz));
  out[4] = fmad(omc, g[4], w1 * (Kr - Vr));
  out[5] = fmad(omc, g[5], w2 * (Kdp + Sp));
  out[6] = fmad(omc, g[6], w2 * (Kdm + Sm));
  out[7] = fmad(omc, g[7], w2 * (Kdp - Sp));
  out[8] = fmad(omc, g[8], w2 * (Kdm - Sm));
}

// psi - psi_ref from psi^2 (FP64).  FP64 storage: the FP64 square root.  FP32 storage: the
// quotient (psi^2 - psi_ref^2) / (psi + psi_ref), whose numerator is formed in FP64 and whose
// denominator needs only FP32 accuracy; the result is as accurate as its FP32 rounding.
__device__ __forceinline__ double psi_shifted(double psi2, double psi_ref, double psi_ref2, double) {
  (void)psi_ref2;
  return __builtin_sqrt(psi2) - psi_ref;
}
__device__ __forceinline__ float psi_shifted(double psi2, double psi_ref, double psi_ref2, float) {
  const float num = (float)(psi2 - psi_ref2);
  const float den = __builtin_amdgcn_sqrtf((float)psi2) + (float)psi_ref;
  return num * recip(__builtin_fmaxf(den, 1e-30f));
}

// Calls f(integral_constant<P>, t0 + P) for P = 0 .. N - 1 while t0 + P < tend.
template <int P, int N, typename F>
__device__ __forceinline__ void unrolled_rows(F& f, int t0, int tend) {
  if constexpr (P < N) {
    if (t0 + P < tend) {
      f(std::integral_constant<int, P>{}, t0 + P);
      unrolled_rows<P + 1, N>(f, t0, tend);
    }
  }
}

// REGF: carry the populations gathered in stage A in registers until the collision instead
// of gathering them again there (fewer loads that miss L2, more registers).
// MID: some instance takes the source h_i at the link midpoint x + c_i/2 (Sec. 2.2) as the
// mean of h_i at the link's two ends: stage D then only forms m0 = -rho u_r / r and 3H of
// its row into a three-row LDS ring, and a fifth stage E collides the row below it with the
// per-direction means (ghost rows across the axis and the wall hold the mirror values:
// m0 and H_z even, H_r odd).  That adds a row to the pipeline and a column to the halo.
template <typename R, int W, bool MOMENTS, bool REGF, bool GUO, bool MID>
__device__ __forceinline__ void run_item(const SweepArgs<R>& g, const WorkItem wi, char* lds, R* hring, R* mring,
                                         int lane) {
  constexpr int HALO = MID ? 7 : 6;  // columns of halo on either side of the output strip
  constexpr int LAG = MID ? 7 : 6;   // rows from the gather to the collision
  const InstDev I = g.inst[wi.inst];
  const int nz = I.nz, nr = I.nr;
  // lanes past the right halo feed nothing: they gather the last halo lane's column (the
  // same lines), so they add no memory traffic
  const unsigned col = (unsigned)wrapi(wi.k0 - HALO + min(lane, wi.ncols + 2 * HALO - 1), nz);
  const unsigned cm = (unsigned)wrapi((int)col - 1, nz), cp = (unsigned)wrapi((int)col + 1, nz);
  const bool out_lane = lane >= HALO && lane < HALO + wi.ncols;
  const int s = wi.s, e = wi.e;
  const int a_lo = max(0, s - LAG), a_hi = min(nr, e + LAG);
  // gathers touch rows a_lo - 1 .. a_hi: the load descriptor is based at row block x0
  const int x0 = max(0, a_lo - 1);
  const long long rs = 9LL * I.pitch;  // elements between row blocks
  const Planes<R> pin = make_planes<R>(g.fin + I.base + (long long)x0 * rs, I.pitch);
  // stores: rows s .. e - 1, from the same row block; the range ends after row e - 1
  const Planes<R> pout = make_planes<R>(g.fout + I.base + (long long)x0 * rs, I.pitch,
                                        (unsigned)(e - x0) * (unsigned)(rs * (long long)sizeof(R)));
  const unsigned bcol = col * (unsigned)sizeof(R), bm = cm * (unsigned)sizeof(R), bp = cp * (unsigned)sizeof(R);
  // The strip that ends a row also fills the row's padding (columns nz .. pitch - 1, never
  // read) from its first halo lanes, so that the row's last line is written whole.
  const int ucol = wi.k0 - HALO + lane;
  const bool pad_lane = wi.k0 + wi.ncols == nz && ucol >= nz && ucol < I.pitch;
  const unsigned bst = pad_lane ? (unsigned)ucol * (unsigned)sizeof(R) : bcol;
  // Other halo lanes (and idle pipeline steps) issue the same stores at an offset past the
  // store descriptor's range, which the hardware drops: every wave then issues the same
  // store sequence, which keeps the compiler's wait counts exact, without writing anything.
  constexpr unsigned kDrop = 0x80000000u;
  const int b_lo = max(0, s - LAG + 2), b_hi = min(nr, e + LAG - 2);
  const int c_lo = max(0, s - LAG + 4), c_hi = min(nr, e + LAG - 4);
  const int d_lo = max(0, s - 1), d_hi = min(nr, e + 1);  // rows of the source ring (MID)
  const R omega = R(I.omega), nu = R(I.nu), gzf = R(I.gz), rho_ref = R(I.rho_ref);
  const R A6 = R(6.0 * I.A), B6 = R(6.0 * (1.0 - 2.0 * I.A));
  const R top_uz = I.bc_top == LBM_TOP_NO_SLIP ? R(-1) : R(1);
  const R psi_ref = R(I.psi_ref), pr2 = R(2.0 * I.psi_ref);
  const bool guo = GUO && I.forcing == LBM_FORCING_GUO;
  const bool mid = MID && I.source_mid != 0;
  // LEAN (FP64 with the populations in registers, node source): F_K travels from stage B to
  // stage C in two more ring fields (in the slot of its row, which no later row takes over
  // before stage C reads it), and kappa and 1/r are computed again where they are used (the
  // same expressions, so the same values): that frees the 24 VGPRs that let the carried
  // populations fit two waves per SIMD (251 VGPRs and 73 KB of LDS at W 256).
  constexpr bool LEAN = REGF && sizeof(R) == 8 && !MID && !MOMENTS;
  constexpr int NF = ring_fields<R, MOMENTS, REGF, MID>();
  const Rings<R, W, NF> L{lds};
  constexpr int ROWB = Rings<R, W, NF>::ROWB;
  constexpr R i36 = R(1.0 / 36.0);

  // rb[k] = this lane's byte offset in the ring slot holding row t - k (slot = row mod 5);
  // stepping t rotates the five offsets by one.  They are carried per lane so that each
  // ring access is a single base register plus an immediate.
  int rb[5];
  const int lane_off = lane * NF * (int)sizeof(R);
#pragma unroll
  for (int k = 0; k < 5; ++k) rb[k] = lane_off + slot(a_lo - k) * ROWB;

  // node values travelling from stage A to stage C (age 4) and to the collision (age LAG),
  // and from B/C onward
  // The row gathered at iteration t sits in slot (t - a_lo) mod PER of fd (and, when the
  // populations are gathered again for the collision, of sg_s, jz_s, jr_s) until its
  // collision LAG iterations later.  The row loop is unrolled PER times so that every slot
  // index is a constant: the carried rows need no register moves, and the next row is
  // gathered straight into its slot (PER = LAG + 2, so that slot is not the one the
  // collision reads).  With the populations in registers (REGF) in FP32 the moments summed
  // in stage A go to this lane's own column of an LDS ring (mring), slot by slot like fd,
  // and stages C and D read them back instead of summing them again: registers alone would
  // not hold them at three waves per SIMD.  No other lane reads them, so no barrier orders
  // them.  FP64 sums them again from the carried populations (the same sums in the same
  // order): its LDS goes to the LEAN ring fields.
  constexpr int PER = LAG + 2;
  constexpr int MS = REGF ? 1 : PER;
  R sg_s[MS], jz_s[MS], jr_s[MS], kap_d[5];
#pragma unroll
  for (int q = 0; q < MS; ++q) sg_s[q] = jz_s[q] = jr_s[q] = R(0);
  auto moments = [](const R* f, R& sg, R& jz, R& jr) {
    sg = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    jz = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
    jr = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
  };
#pragma unroll
  for (int q = 0; q < 5; ++q) kap_d[q] = R(0);
  R fk0z = 0, fk0r = 0, fk1z = 0, fk1r = 0, fk2z = 0, fk2r = 0;
  R fcz[LAG - 3], fcr[LAG - 3];  // F of the stage-C row, carried to the collision
#pragma unroll
  for (int q = 0; q < LAG - 3; ++q) fcz[q] = fcr[q] = R(0);
  R ir0 = 0, ir1 = 0, ir2 = 0;  // 1/r of the stage-C row, two iterations deep
  int bad = 0;

  R fd[REGF ? PER : 1][9];  // populations of the rows in flight (REGF only), by slot
#pragma unroll
  for (int a = 0; a < (REGF ? PER : 1); ++a)
#pragma unroll
    for (int i = 0; i < 9; ++i) fd[a][i] = R(0);

  R fa[9], fg[9];
  // moments of the row in slot sl
  auto mom = [&](int sl, int q) -> R& { return mring[(sl * 3 + q) * W + lane]; };
  auto carried = [&](int sl, R& sg, R& jz, R& jr) {
    if (REGF && sizeof(R) == 4) {
      sg = mom(sl, 0);
      jz = mom(sl, 1);
      jr = mom(sl, 2);
    } else if (REGF) {
      moments(fd[REGF ? sl : 0], sg, jz, jr);
    } else {
      sg = sg_s[REGF ? 0 : sl];
      jz = jz_s[REGF ? 0 : sl];
      jr = jr_s[REGF ? 0 : sl];
    }
  };
  if (a_lo < a_hi) gather_row<R>(pin, nr, I.bc_top, a_lo, x0, bm, bcol, bp, REGF ? fd[0] : fa);
  if (!REGF && !MOMENTS && s < e) gather_row<R>(pin, nr, I.bc_top, s, x0, bm, bcol, bp, fg);
  if (!MOMENTS) {  // the (dropped) stores of a step, so that loop entry looks like a loop iteration
#pragma unroll
    for (int i = 0; i < 9; ++i) bstore(__builtin_nondeterministic_value(R(0)), pout.g, kDrop, i * pout.pstride);
  }

  // Populations of row x for its collision: carried in registers (REGF) or the row gathered
  // one collision ahead, whose successor is gathered now.
  auto take_f = [&](int x, int sl, R f[9]) {
    if (x < s || x >= e) return;
    if (REGF) {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = fd[REGF ? sl : 0][i];
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = fg[i];
      if (x + 1 < e) gather_row<R>(pin, nr, I.bc_top, x + 1, x0, bm, bcol, bp, fg);
    }
  };
  // Collision of row x (eq. lbm) and the nine stores of its populations; h_i enters through
  // m0 and 3H (node source), or per direction through hmid (link-midpoint source, MID).
  auto collide_store = [&](int x, int sl, const R f[9], R m0, R H3z, R H3r, const R* hmid) {
    const bool active = x >= s && x < e;
    R o[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) o[i] = __builtin_nondeterministic_value(R(0));
    if (active) {
      R sg, jz, jr;
      carried(sl, sg, jz, jr);
      const R rho = rho_ref + sg;
      collide<R>(f, rho, sg, jz, jr, fcz[LAG - 4], fcr[LAG - 4], m0, H3z, H3r, omega, guo, o);
      if (MID && hmid) {
#pragma unroll
        for (int i = 0; i < 9; ++i) o[i] += hmid[i];
      }
    }
    // Every iteration issues the same nine stores (dropped while the stage idles and for
    // halo lanes), which lets the compiler keep the prefetched loads in flight.
    const unsigned orow = active ? (unsigned)(x - x0) * pout.rstride : 0u;
    const unsigned voff = active && (out_lane || pad_lane) ? bst : kDrop;
#pragma unroll
    for (int i = 0; i < 9; ++i) bstore(o[i], pout.g, voff, orow + i * pout.pstride);
  };

  auto row = [&](auto Pc, int t) {
    constexpr int P = decltype(Pc)::value;
    constexpr int S0 = P, S1 = (P + 1) % PER;                  // this row's slot, the next row's
    constexpr int S4 = (P + PER - 4) % PER, S6 = (P + PER - 6) % PER, SL = (P + PER - LAG) % PER;
#pragma unroll
    for (int q = 4; q > 0; --q) kap_d[q] = kap_d[q - 1];
    fk2z = fk1z; fk2r = fk1r; fk1z = fk0z; fk1r = fk0r;
#pragma unroll
    for (int q = LAG - 4; q > 0; --q) {
      fcz[q] = fcz[q - 1];
      fcr[q] = fcr[q - 1];
    }
    ir2 = ir1; ir1 = ir0;
    // ------------------------------------------------------------------ A: row t (slot rb[0])
    {
      const int x = t;
      if (x >= a_lo && x < a_hi) {
        const R* f = REGF ? fd[REGF ? S0 : 0] : fa;
        R sg, jz, jr;
        moments(f, sg, jz, jr);
        if (x + 1 < a_hi) gather_row<R>(pin, nr, I.bc_top, x + 1, x0, bm, bcol, bp, REGF ? fd[REGF ? S1 : 0] : fa);
        const double rd = I.rho_ref + (double)sg;  // rho in FP64 for the EOS
        double Pk, kap;
        eos_dev(I, rd, Pk, kap);
        const double psi2 = I.eos == LBM_EOS_IDEAL ? 0.0 : fmad(rd, 1.0 / 3.0, -Pk);
        if (!(rd > 0.0) || !(rd < I.rmax) || !(psi2 >= 0.0)) bad |= ERR_BIT_DOMAIN;
        if (!isfinite(rd)) bad |= ERR_BIT_NONFINITE;  // any non-finite population makes the sum so
        const R psi = psi_shifted(__builtin_fmax(psi2, 0.0), I.psi_ref, I.psi_ref2, R(0));
        L.at(R_PSI, rb[0], 0) = psi;
        if (x == 0) L.at(R_PSI, rb[1], 0) = psi;  // psi is even across the axis: row -1 = row t - 1
        if (x == 1) L.at(R_PSI, rb[3], 0) = psi;  // row -2 = row t - 3
        if (!REGF) {
          sg_s[REGF ? 0 : S0] = sg;
          jz_s[REGF ? 0 : S0] = jz;
          jr_s[REGF ? 0 : S0] = jr;
        } else if (sizeof(R) == 4) {
          mom(S0, 0) = sg;
          mom(S0, 1) = jz;
          mom(S0, 2) = jr;
        }
        if (!LEAN) kap_d[0] = R(kap);
      } else if (a_hi == nr && x == nr) {
        L.at(R_PSI, rb[0], 0) = L.at(R_PSI, rb[1], 0);  // even at the wall: row nr = row nr - 1
      } else if (a_hi == nr && x == nr + 1) {
        L.at(R_PSI, rb[0], 0) = L.at(R_PSI, rb[3], 0);  // row nr + 1 = row nr - 2
      }
    }
    lds_barrier();

    // ------------------------------------------------------------------ B: row t-2 (rows t-4 .. t)
    {
      const int x = t - 2;
      if (x >= b_lo && x < b_hi) {
        const Rows5 r{rb[4], rb[3], rb[2], rb[1], rb[0]};
        const R dz = stencil_dz36(L, R_PSI, r) * i36;
        const R dr = stencil_dr36(L, R_PSI, r) * i36;
        // F_K = 6 [A sum_i w_i psi_i^2 c_i + (1 - 2A) psi sum_i w_i psi_i c_i], i = 1, 2, ..., 8
        const R w1 = R(1.0 / 9.0), w2 = R(1.0 / 36.0);
        const R q1 = L.at(R_PSI, r.s0, 1), q2 = L.at(R_PSI, r.p1, 0), q3 = L.at(R_PSI, r.s0, -1);
        const R q4 = L.at(R_PSI, r.m1, 0), q5 = L.at(R_PSI, r.p1, 1), q6 = L.at(R_PSI, r.p1, -1);
        const R q7 = L.at(R_PSI, r.m1, -1), q8 = L.at(R_PSI, r.m1, 1);
        const R s1z = w1 * (q1 - q3) + w2 * ((q5 - q7) + (q8 - q6));
        const R s1r = w1 * (q2 - q4) + w2 * ((q5 - q7) - (q8 - q6));
        // psi_i^2 = psi_ref^2 + d_i (2 psi_ref + d_i); the constant cancels in sum_i w_i c_i
        const R t1 = q1 * (pr2 + q1), t2 = q2 * (pr2 + q2), t3 = q3 * (pr2 + q3), t4 = q4 * (pr2 + q4);
        const R t5 = q5 * (pr2 + q5), t6 = q6 * (pr2 + q6), t7 = q7 * (pr2 + q7), t8 = q8 * (pr2 + q8);
        const R s2z = w1 * (t1 - t3) + w2 * ((t5 - t7) + (t8 - t6));
        const R s2r = w1 * (t2 - t4) + w2 * ((t5 - t7) - (t8 - t6));
        const R bpsi = B6 * (psi_ref + L.at(R_PSI, r.s0, 0));
        if (LEAN) {
          L.at(R_FKZ, r.s0, 0) = fmad(A6, s2z, bpsi * s1z);
          L.at(R_FKR, r.s0, 0) = fmad(A6, s2r, bpsi * s1r);
        } else {
          fk0z = fmad(A6, s2z, bpsi * s1z);
          fk0r = fmad(A6, s2r, bpsi * s1r);
        }
        L.at(R_DZ, r.s0, 0) = dz;
        L.at(R_DR, r.s0, 0) = dr;
        if (x == 0) { L.at(R_DZ, rb[3], 0) = dz; L.at(R_DR, rb[3], 0) = -dr; }  // row -1 = row t - 3
        if (x == 1) { L.at(R_DZ, rb[0], 0) = dz; L.at(R_DR, rb[0], 0) = -dr; }  // row -2 = row t - 5
      } else if (b_hi == nr && x == nr) {  // D_z psi even, D_r psi odd at the wall
        L.at(R_DZ, rb[2], 0) = L.at(R_DZ, rb[3], 0);
        L.at(R_DR, rb[2], 0) = -L.at(R_DR, rb[3], 0);
      } else if (b_hi == nr && x == nr + 1) {
        L.at(R_DZ, rb[2], 0) = L.at(R_DZ, rb[0], 0);
        L.at(R_DR, rb[2], 0) = -L.at(R_DR, rb[0], 0);
      }
    }
    lds_barrier();

    // ------------------------------------------------------------------ C: row t-4 (rows t-6 .. t-2)
    {
      const int x = t - 4;
      if (x >= c_lo && x < c_hi) {
        const Rows5 r{rb[1], rb[0], rb[4], rb[3], rb[2]};
        R sg4, jz, jr;
        carried(S4, sg4, jz, jr);
        const R rho = rho_ref + sg4;
        R kap = kap_d[4];
        if (LEAN) {
          double Pk_, kap_;
          eos_dev(I, I.rho_ref + (double)sg4, Pk_, kap_);
          kap = R(kap_);
        }
        R fz = LEAN ? L.at(R_FKZ, r.s0, 0) : fk2z, fr = LEAN ? L.at(R_FKR, r.s0, 0) : fk2r;
        if (I.axisym) {
          // F_axis = 3K/r [psi D_rz psi + 6A D_r psi D_z psi, psi (D_rr psi - D_r psi / r) + 6A (D_r psi)^2]
          const R drr = stencil_dr36(L, R_DR, r) * i36;
          const R drz = stencil_dr36(L, R_DZ, r) * i36;
          const R psi = psi_ref + L.at(R_PSI, r.s0, 0), dz = L.at(R_DZ, r.s0, 0), dr = L.at(R_DR, r.s0, 0);
          const R ir = recip(R(x) + R(0.5));  // 1/r_j (uniform), carried on to stage D unless LEAN
          ir0 = ir;
          const R k3 = (I.faxis_sound ? R(1.0 / 3.0) : R(3) * kap * kap) * ir;
          const R a6dr = A6 * dr;
          fz = fmad(k3, fmad(psi, drz, a6dr * dz), fz);
          fr = fmad(k3, fmad(psi, fmad(-dr, ir, drr), a6dr * dr), fr);
        }
        fz += gzf;
        const R irho = recip(rho);
        const R uz = fmad(R(0.5), fz, jz) * irho;
        const R ur = fmad(R(0.5), fr, jr) * irho;
        fcz[0] = fz;
        fcr[0] = fr;
        L.at(R_UZ, r.s0, 0) = uz;
        L.at(R_UR, r.s0, 0) = ur;
        if (x == 0) { L.at(R_UZ, rb[0], 0) = uz; L.at(R_UR, rb[0], 0) = -ur; }  // row -1 = row t - 5
        if (x == 1) { L.at(R_UZ, rb[2], 0) = uz; L.at(R_UR, rb[2], 0) = -ur; }  // row -2 = row t - 7
        if (MOMENTS && out_lane && x >= s && x < e) {
          const long long o = (long long)x * nz + col;
          g.mrho[o] = (double)rho;
          g.muz[o] = (double)uz;
          g.mur[o] = (double)ur;
        }
      } else if (c_hi == nr && x == nr) {  // u_r odd; u_z even (free slip) or odd (no slip)
        L.at(R_UZ, rb[4], 0) = top_uz * L.at(R_UZ, rb[0], 0);
        L.at(R_UR, rb[4], 0) = -L.at(R_UR, rb[0], 0);
      } else if (c_hi == nr && x == nr + 1) {
        L.at(R_UZ, rb[4], 0) = top_uz * L.at(R_UZ, rb[2], 0);
        L.at(R_UR, rb[4], 0) = -L.at(R_UR, rb[2], 0);
      }
    }
    lds_barrier();

    // ------------------------------------------------------------------ D: row t-6 (rows t-8 .. t-4)
    if (!MOMENTS) {
      const int x = t - 6;
      // H of eq. (axihz) from the velocity ring; H_r carries -u_r/r so that sum_i c_ir h_i
      // supplies C_r = 2 mu d/dr(u_r/r)
      R m0 = R(0), H3z = R(0), H3r = R(0);
      const bool hrow = MID ? (x >= d_lo && x < d_hi) : (x >= s && x < e);
      R f[9];
      if (!MID) take_f(x, SL, f);
      if (I.axisym && hrow) {
        const Rows5 r{rb[3], rb[2], rb[1], rb[0], rb[4]};
        R sg6, jz6, jr6;
        carried(S6, sg6, jz6, jr6);
        const R rho = rho_ref + sg6;
        const R uz = L.at(R_UZ, r.s0, 0), ur = L.at(R_UR, r.s0, 0);
        const R druz = stencil_dr36(L, R_UZ, r);  // 36 D_r u_z
        const R dzur = stencil_dz36(L, R_UR, r);  // 36 D_z u_r
        const R drur = stencil_dr36(L, R_UR, r);  // 36 D_r u_r
        const R ir = LEAN ? recip(R(x) + R(0.5)) : ir2;
        const R mu36 = rho * nu * i36;
        const R ir3 = R(3) * ir;
        const R rur = rho * ur;
        H3z = fmad(mu36, druz + dzur, -rur * uz) * ir3;
        H3r = fmad(R(2) * mu36, fmad(R(-36) * ur, ir, drur), -rur * ur) * ir3;
        m0 = -rur * ir;
      }
      if (!MID) {
        collide_store(x, SL, f, m0, H3z, H3r, nullptr);
      } else {
        // the source ring: element (row slot, column, field), fields m0, 3H_z, 3H_r; the
        // row below the axis and the row beyond the wall hold the mirror values
        auto H = [&](int row, int dz, int q) -> R& {
          return hring[((wrapi(row, 3) * (W + 2)) + lane + 1 + dz) * 3 + q];
        };
        if (hrow) {
          H(x, 0, 0) = m0;
          H(x, 0, 1) = H3z;
          H(x, 0, 2) = H3r;
          if (x == 0) { H(-1, 0, 0) = m0; H(-1, 0, 1) = H3z; H(-1, 0, 2) = -H3r; }
        } else if (d_hi == nr && x == nr) {
          H(nr, 0, 0) = H(nr - 1, 0, 0);
          H(nr, 0, 1) = H(nr - 1, 0, 1);
          H(nr, 0, 2) = -H(nr - 1, 0, 2);
        }
        lds_barrier();
        // ---------------------------------------------------------------- E: row t-7 (rows t-8 .. t-6)
        const int xe = t - 7;
        take_f(xe, SL, f);
        if (!mid) {
          collide_store(xe, SL, f, H(xe, 0, 0), H(xe, 0, 1), H(xe, 0, 2), nullptr);
        } else {
          // h_i(x + c_i/2) = (h_i(x) + h_i(x + c_i)) / 2, h_i = w_i (m0 + c_iz 3H_z + c_ir 3H_r)
          const R w0 = R(4.0 / 9.0), w1 = R(1.0 / 18.0), w2 = R(1.0 / 72.0);  // w_i / 2 for i > 0
          const R a0 = H(xe, 0, 0), az = H(xe, 0, 1), ar = H(xe, 0, 2);
          auto link = [&](int dr, int dz, R wh, int cz, int cr) {
            const R b0 = H(xe + dr, dz, 0), bz = H(xe + dr, dz, 1), bhr = H(xe + dr, dz, 2);
            return wh * ((a0 + b0) + R(cz) * (az + bz) + R(cr) * (ar + bhr));
          };
          R hm[9];
          hm[0] = w0 * a0;
          hm[1] = link(0, 1, w1, 1, 0);
          hm[2] = link(1, 0, w1, 0, 1);
          hm[3] = link(0, -1, w1, -1, 0);
          hm[4] = link(-1, 0, w1, 0, -1);
          hm[5] = link(1, 1, w2, 1, 1);
          hm[6] = link(1, -1, w2, -1, 1);
          hm[7] = link(-1, -1, w2, -1, -1);
          hm[8] = link(-1, 1, w2, 1, -1);
          collide_store(xe, SL, f, R(0), R(0), R(0), hm);
        }
      }
    }
    {  // row t + 1 takes the slot of row t - 4
      const int r4 = rb[4];
      rb[4] = rb[3];
      rb[3] = rb[2];
      rb[2] = rb[1];
      rb[1] = rb[0];
      rb[0] = r4;
    }
  };
  for (int t0 = a_lo; t0 < e + LAG; t0 += PER) unrolled_rows<0, PER>(row, t0, e + LAG);
  if (bad) {
    atomicOr(g.err, bad);                 // any instance
    atomicOr(g.err + 1 + wi.inst, bad);   // this instance
  }
}

__device__ __forceinline__ int xcd_map(int b, int G) {
  // Hardware hands workgroup b to XCD b % 8; give each XCD one contiguous run of items.
  const int xcd = b & 7, pos = b >> 3;
  const int q = G >> 3, rem = G & 7;
  return xcd < rem ? xcd * (q + 1) + pos : rem * (q + 1) + (xcd - rem) * q + pos;
}

// Minimum waves per SIMD asked of the register allocator (168 VGPRs for three waves, 256 for
// two): three in FP32, two in FP64 (with the populations in registers, FP64 fits two only
// through run_item's LEAN form).  The budget must not force spills: a spill reload goes
// through the vector memory counter and would make the wave wait for its prefetched rows.
// The persistent loop keeps more state live: one wave less.  The link-midpoint source (MID)
// keeps more values live: in FP32 two waves with the populations in registers, three when
// gathering again (two for the persistent loop); in FP64 one.
template <typename R, bool PERSIST, bool REGF, bool MID>
struct SweepWaves {
  static constexpr int base = sizeof(R) == 4 ? 3 : 2;
  static constexpr int mid = sizeof(R) == 8 ? 1 : REGF ? 2 : PERSIST ? 2 : 3;
  static constexpr int value = MID ? mid : PERSIST ? base - 1 : base;
};

// GUO: some instance of the launch uses Guo's forcing (a per-instance branch); otherwise
// only the exact-difference collision is compiled in.  MID: some instance takes its source
// at the link midpoint (the deeper pipeline of run_item); otherwise the node source only.
template <typename R, int W, bool MOMENTS, bool PERSIST, bool REGF, bool GUO, bool MID>
__global__ void __launch_bounds__(W)
__attribute__((amdgpu_waves_per_eu(SweepWaves<R, PERSIST, REGF, MID>::value))) k_sweep(SweepArgs<R> g) {
  constexpr int HALO = MID ? 7 : 6;
  __shared__ R ring[RD][W + 4][ring_fields<R, MOMENTS, REGF, MID>()];
  __shared__ R hring[MID ? 3 * (W + 2) * 3 : 1];
  __shared__ R mring[REGF && !MOMENTS && sizeof(R) == 4 ? (MID ? 9 : 8) * 3 * W : 1];  // moments, slot by slot
  __shared__ int s_ticket;
  const int lane = threadIdx.x;
  char* const lds = reinterpret_cast<char*>(&ring[0][0][0]);
  if (!PERSIST) {
    const int b = (int)blockIdx.x;
    const int item = g.xcd_swizzle ? xcd_map(b, (int)gridDim.x) : b;
    if (item >= g.n_items) return;
    const WorkItem wi = g.items[item];
    // Only lanes 0 .. ncols + 2 HALO - 1 (the output columns and the halo columns on either
    // side) feed an output, and at the end of a row the lanes that fill its padding store.  A
    // wave with none of them ends here, which frees its SIMD slot for other workgroups (narrow
    // members of a batch, the last strip of a row); s_barrier waits only for the waves of
    // the group still running.
    const InstDev* ip = g.inst + wi.inst;
    const int need = wi.k0 + wi.ncols == ip->nz ? max(wi.ncols + 2 * HALO, ip->pitch - wi.k0 + HALO)
                                                : wi.ncols + 2 * HALO;
    if (__builtin_amdgcn_readfirstlane(lane >> 6) * 64 >= need) return;
    run_item<R, W, MOMENTS, REGF, GUO, MID>(g, wi, lds, hring, mring, lane);
    return;
  }
  for (;;) {
    if (lane == 0) s_ticket = atomicAdd(&g.queue[0], 1);
    lds_barrier();
    const int item = __builtin_amdgcn_readfirstlane(s_ticket);  // uniform across the workgroup
    lds_barrier();
    if (item >= g.n_items) break;
    run_item<R, W, MOMENTS, REGF, GUO, MID>(g, g.items[item], lds, hring, mring, lane);
  }
  if (lane == 0) {
    // The last workgroup out rewinds the queue for the next launch (no memset needed,
    // which keeps graph replays free of memset nodes).
    const int done = atomicAdd(&g.queue[1], 1);
    if (done == (int)gridDim.x - 1) {
      atomicExch(&g.queue[0], 0);
      atomicExch(&g.queue[1], 0);
    }
  }
}

// ---------------------------------------------------------------------------- init / checkpoint

__device__ __constant__ int c_cz[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ __constant__ int c_cr[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ __constant__ int c_mirror_r[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};  // (c_z, c_r) -> (c_z, -c_r)
__device__ __constant__ int c_opposite[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};  // c -> -c

// Post-collision planes whose streaming yields the given post-streaming state f0:
// the inverse of the pull map.  f0 is either a double [9][nr][nz] array, or (when
// f0 == nullptr) the equilibrium E(rho0, u0) of the initial fields (Sec. 2.1).
template <typename R>
__global__ void k_unstream(R* __restrict__ fout, int nz, int pitch, int nr, int bc_top, double rho_ref,
                           const double* __restrict__ rho0, const double* __restrict__ uz0,
                           const double* __restrict__ ur0, const double* __restrict__ f0) {
  const double wgt[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                         1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  const long long n = (long long)nz * nr;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n;
       id += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(id % nz), j = (int)(id / nz);
    for (int i = 0; i < 9; ++i) {
      int tk = k + c_cz[i], tj = j + c_cr[i], ti = i;
      if (tj < 0) {
        tj = 0;
        ti = c_mirror_r[i];
      } else if (tj >= nr) {
        tj = nr - 1;
        if (bc_top == LBM_TOP_NO_SLIP) {
          tk = k;
          ti = c_opposite[i];
        } else {
          ti = c_mirror_r[i];
        }
      }
      tk = wrapi(tk, nz);
      const long long tn = (long long)tj * nz + tk;
      double v;
      if (f0) {
        v = f0[ti * n + tn] - wgt[ti] * rho_ref;
      } else {
        double e[9];
        shifted_equilibrium<double>(rho0[tn], rho0[tn] - rho_ref, uz0 ? uz0[tn] : 0.0,
                                    ur0 ? ur0[tn] : 0.0, e);
        v = e[ti];
      }
      fout[(9LL * j + i) * pitch + k] = R(v);
    }
  }
}

template <typename R>
__global__ void k_export(const R* __restrict__ fin, int nz, int pitch, int nr, int bc_top, double rho_ref,
                         double* __restrict__ out) {
  const double wgt[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                         1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  const long long n = (long long)nz * nr;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n;
       id += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(id % nz), j = (int)(id / nz);
    R f[9];
    gather<R>(fin, pitch, nr, bc_top, j, (unsigned)wrapi(k - 1, nz), (unsigned)k, (unsigned)wrapi(k + 1, nz), f);
    for (int i = 0; i < 9; ++i) out[i * n + id] = (double)f[i] + wgt[i] * rho_ref;
  }
}

// ---------------------------------------------------------------------------- reductions

// Fixed-shape FP64 block reduction (64-lane wavefronts, then LDS): deterministic.
template <int NT, int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double (*sm)[K]) {
#pragma unroll
  for (int q = 0; q < K; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0)
    for (int q = 0; q < K; ++q) sm[w][q] = v[q];
  lds_barrier();
  if (threadIdx.x == 0) {
    for (int q = 0; q < K; ++q) {
      double s = 0.0;
      for (int i = 0; i < NT / 64; ++i) s += sm[i][q];
      v[q] = s;
    }
  }
}


// Per row: K = 1: sum_k rho; K = 4: (sum P_k, count) inside r_in and (sum P_k, count) beyond r_out.
template <typename R, int K>
__global__ void __launch_bounds__(256) k_rows(const R* __restrict__ fin,
                                              const InstDev* __restrict__ inst,
                                              const RowRef* __restrict__ rows,
                                              const double* __restrict__ geo, double* __restrict__ part) {
  __shared__ double sm[4][K];
  const RowRef rr = rows[blockIdx.x];
  const InstDev I = inst[rr.inst];
  const int nz = I.nz, j = rr.row;
  const R* f = fin + I.base;
  double acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0;
  const double rj = j + 0.5;
  for (int k = threadIdx.x; k < nz; k += 256) {
    R o[9];
    gather<R>(f, I.pitch, I.nr, I.bc_top, j, (unsigned)wrapi(k - 1, nz), (unsigned)k, (unsigned)wrapi(k + 1, nz), o);
    const R sg = o[0] + o[1] + o[2] + o[3] + o[4] + o[5] + o[6] + o[7] + o[8];
    const double rho = I.rho_ref + (double)sg;
    if (K == 1) {
      acc[0] += rho;
    } else {
      const double zc = geo[3 * rr.inst], rin = geo[3 * rr.inst + 1], rout = geo[3 * rr.inst + 2];
      double Pk, kap;
      eos_dev(I, rho, Pk, kap);
      const double d = sqrt((k - zc) * (k - zc) + rj * rj);
      if (d < rin) {
        acc[0] += Pk;
        acc[1] += 1.0;
      }
      if (d > rout) {
        acc[2] += Pk;
        acc[3] += 1.0;
      }
    }
  }
  block_sum<256, K>(acc, sm);
  if (threadIdx.x == 0)
    for (int q = 0; q < K; ++q) part[(long long)blockIdx.x * K + q] = acc[q];
}

// Sec. 3.2 follows the oscillating drop by where its interface crosses the symmetry axis.
// One workgroup per instance: on the axis row, k* = the smallest k >= floor(zc) whose next
// node has rho_{k+1} <= thr, then z = k* + (rho_k* - thr) / (rho_k* - rho_{k*+1}); NaN when
// no column before the last qualifies.
template <typename R>
__global__ void __launch_bounds__(256) k_axis(const R* __restrict__ fin, const InstDev* __restrict__ inst,
                                              const double* __restrict__ geo, double* __restrict__ out) {
  __shared__ int s_k;
  const int n = blockIdx.x;
  const InstDev I = inst[n];
  const int nz = I.nz;
  const R* f = fin + I.base;
  const double thr = geo[2 * n + 1];
  const int k0 = (int)floor(geo[2 * n]);
  auto rho_at = [&](int k) {
    R o[9];
    gather<R>(f, I.pitch, I.nr, I.bc_top, 0, (unsigned)wrapi(k - 1, nz), (unsigned)k, (unsigned)wrapi(k + 1, nz), o);
    const R sg = o[0] + o[1] + o[2] + o[3] + o[4] + o[5] + o[6] + o[7] + o[8];
    return I.rho_ref + (double)sg;
  };
  if (threadIdx.x == 0) s_k = 0x7fffffff;
  __syncthreads();
  int best = 0x7fffffff;
  for (int k = k0 + (int)threadIdx.x; k + 1 < nz; k += 256)
    if (rho_at(k + 1) <= thr) {  // the first hit of this lane's stride is its smallest
      best = k;
      break;
    }
  atomicMin(&s_k, best);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int k = s_k;
    if (k == 0x7fffffff) {
      out[n] = __builtin_nan("");
    } else {
      const double rk = rho_at(k), rn = rho_at(k + 1);
      out[n] = k + (rk - thr) / (rk - rn);
    }
  }
}

// Per instance: combine its rows' partials in a fixed order.
template <int K>
__global__ void __launch_bounds__(256) k_finish(const double* __restrict__ part,
                                                const int* __restrict__ row_start,
                                                const InstDev* __restrict__ inst, double* __restrict__ out) {
  __shared__ double sm[4][K];
  const int n = blockIdx.x;
  const int r0 = row_start[n], r1 = row_start[n + 1];
  double acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0;
  for (int r = r0 + threadIdx.x; r < r1; r += 256) {
    if (K == 1) {
      const double rj = (r - r0) + 0.5;
      acc[0] += 2.0 * M_PI * rj * part[r];
    } else {
      for (int q = 0; q < K; ++q) acc[q] += part[(long long)r * K + q];
    }
  }
  block_sum<256, K>(acc, sm);
  if (threadIdx.x == 0) {
    if (K == 1)
      out[n] = acc[0];
    else
      out[n] = (acc[1] > 0.0 && acc[3] > 0.0) ? acc[0] / acc[1] - acc[2] / acc[3] : __builtin_nan("");
  }
  (void)inst;
}

// ---------------------------------------------------------------------------- copy (bandwidth reference)

// Plain streaming copy: one 16-byte access per lane, one workgroup per consecutive 4 KiB, so
// the workgroups in flight sweep a compact address window.  (Measured faster than a
// grid-stride loop, whose workgroups drift apart.)  Used to measure the practical HBM copy
// rate and to calibrate the byte counters of the profiler.
__global__ void __launch_bounds__(256) k_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                              long long n16) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

hipError_t launch_copy(const void* src, void* dst, long long bytes, hipStream_t st) {
  const long long blocks = (bytes / 16 + 255) / 256;
  if (blocks < 1 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<const float4*>(src),
                     static_cast<float4*>(dst), bytes / 16);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------- host-side launchers

template <typename R, int W, bool MOMENTS, bool PERSIST, bool REGF, bool GUO, bool MID>
static hipError_t launch_sweep(const SweepArgs<R>& g, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_sweep<R, W, MOMENTS, PERSIST, REGF, GUO, MID>), dim3(grid), dim3(W), 0, st, g);
  return hipGetLastError();
}

template <typename R, int W, bool GUO, bool MID>
static hipError_t launch_step(const SweepArgs<R>& g, bool persist, bool regf, int grid, hipStream_t st) {
  if (persist)
    return regf ? launch_sweep<R, W, false, true, true, GUO, MID>(g, grid, st)
                : launch_sweep<R, W, false, true, false, GUO, MID>(g, grid, st);
  return regf ? launch_sweep<R, W, false, false, true, GUO, MID>(g, grid, st)
              : launch_sweep<R, W, false, false, false, GUO, MID>(g, grid, st);
}

// The link-midpoint kernels carry Guo's per-instance branch too (one instantiation for both).
template <typename R>
hipError_t sweep_dispatch(const SweepArgs<R>& g, int width, bool moments, bool persist, bool regf, bool guo,
                          bool mid, int grid, hipStream_t st) {
#define LBM_CASE(WW)                                                                                \
  case WW:                                                                                          \
    if (moments) return launch_sweep<R, WW, true, false, false, false, false>(g, grid, st);         \
    if (mid) return launch_step<R, WW, true, true>(g, persist, regf, grid, st);                     \
    return guo ? launch_step<R, WW, true, false>(g, persist, regf, grid, st)                        \
               : launch_step<R, WW, false, false>(g, persist, regf, grid, st);
  switch (width) {
    LBM_CASE(64)
    LBM_CASE(128)
    LBM_CASE(256)
    default:
      break;
  }
#undef LBM_CASE
  return hipErrorInvalidValue;
}

template hipError_t sweep_dispatch<float>(const SweepArgs<float>&, int, bool, bool, bool, bool, bool, int,
                                          hipStream_t);
template hipError_t sweep_dispatch<double>(const SweepArgs<double>&, int, bool, bool, bool, bool, bool, int,
                                           hipStream_t);

template <typename R>
hipError_t launch_unstream(R* fout, int nz, int pitch, int nr, int bc_top, double rho_ref, const double* rho0,
                           const double* uz0, const double* ur0, const double* f0, hipStream_t st) {
  const long long n = (long long)nz * nr;
  const int grid = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
  hipLaunchKernelGGL((k_unstream<R>), dim3(grid), dim3(256), 0, st, fout, nz, pitch, nr, bc_top, rho_ref,
                     rho0, uz0, ur0, f0);
  return hipGetLastError();
}
template hipError_t launch_unstream<float>(float*, int, int, int, int, double, const double*, const double*,
                                           const double*, const double*, hipStream_t);
template hipError_t launch_unstream<double>(double*, int, int, int, int, double, const double*, const double*,
                                            const double*, const double*, hipStream_t);

template <typename R>
hipError_t launch_export(const R* fin, int nz, int pitch, int nr, int bc_top, double rho_ref, double* out,
                         hipStream_t st) {
  const long long n = (long long)nz * nr;
  const int grid = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
  hipLaunchKernelGGL((k_export<R>), dim3(grid), dim3(256), 0, st, fin, nz, pitch, nr, bc_top, rho_ref, out);
  return hipGetLastError();
}
template hipError_t launch_export<float>(const float*, int, int, int, int, double, double*, hipStream_t);
template hipError_t launch_export<double>(const double*, int, int, int, int, double, double*, hipStream_t);

template <typename R>
hipError_t launch_rows(int K, const R* fin, const InstDev* inst, const RowRef* rows, int nrows,
                       const double* geo, double* part, hipStream_t st) {
  if (K == 1)
    hipLaunchKernelGGL((k_rows<R, 1>), dim3(nrows), dim3(256), 0, st, fin, inst, rows, geo, part);
  else
    hipLaunchKernelGGL((k_rows<R, 4>), dim3(nrows), dim3(256), 0, st, fin, inst, rows, geo, part);
  return hipGetLastError();
}
template hipError_t launch_rows<float>(int, const float*, const InstDev*, const RowRef*, int, const double*,
                                       double*, hipStream_t);
template hipError_t launch_rows<double>(int, const double*, const InstDev*, const RowRef*, int, const double*,
                                        double*, hipStream_t);

template <typename R>
hipError_t launch_axis(const R* fin, const InstDev* inst, int n, const double* geo, double* out, hipStream_t st) {
  hipLaunchKernelGGL((k_axis<R>), dim3(n), dim3(256), 0, st, fin, inst, geo, out);
  return hipGetLastError();
}
template hipError_t launch_axis<float>(const float*, const InstDev*, int, const double*, double*, hipStream_t);
template hipError_t launch_axis<double>(const double*, const InstDev*, int, const double*, double*, hipStream_t);

hipError_t launch_finish(int K, const double* part, const int* row_start, const InstDev* inst, int n,
                         double* out, hipStream_t st) {
  if (K == 1)
    hipLaunchKernelGGL((k_finish<1>), dim3(n), dim3(256), 0, st, part, row_start, inst, out);
  else
    hipLaunchKernelGGL((k_finish<4>), dim3(n), dim3(256), 0, st, part, row_start, inst, out);
  return hipGetLastError();
}

}  // namespace lbm
