// Host side of the C ABI in lbm_axi.h: argument checks, device memory layout,
// work lists, launches, hipGraph chunks and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "lbm_axi.h"
#include "lbm_axi_internal.h"
#include "scratch.h"
#include "work_items.h"

using namespace lbm;

struct lbm_axi_s {
  int n = 0;
  int prec = LBM_PREC_FP64;
  std::vector<lbm_axi_params> prm;
  std::vector<InstDev> hinst;
  std::vector<long long> base;
  long long felems = 0;  // elements of one distribution buffer (all instances, padded)
  long long nodes = 0;  // real nodes
  size_t esize = 8;
  int device = 0;  // the device current at set-up, whose stream and memory the handle uses
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  void* fbuf[2] = {nullptr, nullptr};
  bool own_f = false;
  int cur = 0;  // fbuf[cur] holds the post-collision planes of the last step
  InstDev* d_inst = nullptr;
  WorkItem* d_items = nullptr;
  int n_items = 0;
  size_t items_cap = 0;
  int* d_queue = nullptr;
  int* d_err = nullptr;
  RowRef* d_rows = nullptr;
  int* d_row_start = nullptr;
  int n_rows = 0;
  double* d_part = nullptr;
  double* d_out = nullptr;
  double* d_geo = nullptr;
  lbm_axi_launch launch{};
  int cus = 256;
  int graph_chunk = 0;
  bool any_guo = false;  // some instance uses Guo's forcing: launch the kernel that can apply it
  bool any_mid = false;  // some instance takes its source at the link midpoint: the deeper pipeline
  // Stream groups: with launch.streams > 1 the instances of a batch are split into groups,
  // each stepped by launches of its own on a stream of its own (group 0 on `stream`), so that
  // the last work items of one group's step overlap the next step of the others.  Steps fork
  // from and join back into `stream`, which every other operation of the handle uses.
  struct Group {
    hipStream_t st = nullptr;  // group 0: the handle's stream (not owned by the group)
    hipEvent_t done = nullptr;
    int first = 0, count = 0;  // the group's work items in d_items
    hipGraphExec_t gexec[2] = {nullptr, nullptr};  // graph_chunk steps starting from fbuf[0] / fbuf[1]
  };
  Group grp[kMaxStreams];
  int n_groups = 1;
  hipEvent_t fork = nullptr;
  // Moments: one instance's three fields and every instance's work list of the moments
  // launch (at the current strip width and segment length), set up on first use.
  double* d_mom = nullptr;
  WorkItem* d_mitems = nullptr;
  std::vector<int> mfirst, mcount;
  int m_width = 0, m_seg = -1;
};

namespace {

#define HIPCHK(call)                             \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return LBM_ERR_HIP;    \
  } while (0)

lbm_status check_params(const lbm_axi_params& p) {
  if (p.nz < 1 || p.nr < 4) return LBM_ERR_ARG;
  if ((long long)p.nz * p.nr > (1LL << 31)) return LBM_ERR_ARG;
  if (!(p.tau > 0.5) || !std::isfinite(p.tau)) return LBM_ERR_ARG;
  if (p.eos < LBM_EOS_IDEAL || p.eos > LBM_EOS_CS) return LBM_ERR_ARG;
  if (p.eos == LBM_EOS_CS && !(p.eos_b > 0.0)) return LBM_ERR_ARG;
  if (p.eos != LBM_EOS_IDEAL && !(p.lambda > 0.0)) return LBM_ERR_ARG;
  if (p.bc_top != LBM_TOP_FREE_SLIP && p.bc_top != LBM_TOP_NO_SLIP) return LBM_ERR_ARG;
  if (p.axisym != 0 && p.axisym != 1) return LBM_ERR_ARG;
  if (p.faxis_sound != 0 && p.faxis_sound != 1) return LBM_ERR_ARG;
  if (p.forcing != LBM_FORCING_EDM && p.forcing != LBM_FORCING_GUO) return LBM_ERR_ARG;
  if (p.source_mid != 0 && p.source_mid != 1) return LBM_ERR_ARG;
  if (!std::isfinite(p.A) || !std::isfinite(p.gz) || !std::isfinite(p.T)) return LBM_ERR_ARG;
  return LBM_OK;
}

// Host check that an initial density field lies in the EOS domain (psi real), so that a
// bad input is refused before anything is launched.
lbm_status check_rho0(const lbm_axi_params& p, const double* rho) {
  const long long n = (long long)p.nz * p.nr;
  for (long long x = 0; x < n; ++x) {
    const double r = rho[x];
    if (!std::isfinite(r)) return LBM_ERR_NONFINITE;
    if (!(r > 0.0)) return LBM_ERR_EOS_DOMAIN;
    if (p.eos == LBM_EOS_IDEAL) continue;
    double P;
    if (p.eos == LBM_EOS_VDW) {
      if (!(r < 3.0)) return LBM_ERR_EOS_DOMAIN;
      P = p.lambda * (8.0 * r * p.T / (3.0 - r) - 3.0 * r * r);
    } else {
      const double e = 0.25 * p.eos_b * r;
      if (!(e < 1.0)) return LBM_ERR_EOS_DOMAIN;
      const double m = 1.0 - e;
      P = p.lambda * (p.eos_R * p.T * r * (1.0 + e * (1.0 + e * (1.0 - e))) / (m * m * m) - p.eos_a * r * r);
    }
    if (!(r / 3.0 - P >= 0.0)) return LBM_ERR_EOS_DOMAIN;
  }
  return LBM_OK;
}

// Storage reference density of an FP32 instance: the median of (a sample of) its initial
// density, i.e. the density of the phase that fills most of the domain.
double reference_density(const lbm_axi_params& p, const double* rho0) {
  const long long n = (long long)p.nz * p.nr;
  const long long stride = std::max(1LL, n / 1000003);
  std::vector<double> s;
  for (long long x = 0; x < n; x += stride) s.push_back(rho0[x]);
  std::nth_element(s.begin(), s.begin() + s.size() / 2, s.end());
  return s[s.size() / 2];
}

InstDev make_inst(const lbm_axi_params& p, long long base, double rho_ref, int esize) {
  InstDev d{};
  d.rho_ref = rho_ref;
  d.psi_ref = rho_ref > 0.0 ? eos_psi(p, rho_ref) : 0.0;
  d.base = base;
  d.nz = p.nz;
  d.nr = p.nr;
  d.pitch = row_pitch(p.nz, esize);
  d.eos = p.eos;
  d.axisym = p.axisym;
  d.faxis_sound = p.faxis_sound;
  d.bc_top = p.bc_top;
  d.forcing = p.forcing;
  d.source_mid = p.source_mid;
  d.psi_ref2 = d.psi_ref * d.psi_ref;
  if (p.eos == LBM_EOS_CS) {
    d.c1 = p.lambda * p.eos_R * p.T;
    d.c2 = p.lambda * p.eos_a;
    d.ce = 0.25 * p.eos_b;
    d.rmax = 4.0 / p.eos_b;
  } else if (p.eos == LBM_EOS_VDW) {
    d.c1 = 8.0 * p.lambda * p.T;
    d.c2 = 3.0 * p.lambda;
    d.ce = 0.0;
    d.rmax = 3.0;
  } else {
    d.c1 = d.c2 = d.ce = 0.0;
    d.rmax = HUGE_VAL;
  }
  d.A = p.A;
  d.omega = 1.0 / p.tau;
  d.nu = (p.tau - 0.5) / 3.0;
  d.gz = p.gz;
  return d;
}

bool valid_width(int w) { return w == 64 || w == 128 || w == 256; }

// Default shape without timing anything: minimise max(total lane-iterations / lanes the chip
// keeps in flight, longest item / 3), the second term being the chain of one work item when
// the chip is under-filled (its waves then run about three times faster).  The populations
// ride in registers (fewer bytes, the same results), except in FP64 with the link-midpoint
// source, whose register form fits only one wave per SIMD.
lbm_axi_launch default_launch(const lbm_axi_s* h) {
  const int regf = h->prec == LBM_PREC_FP32 || !h->any_mid ? 1 : 0;
  lbm_axi_launch best{};
  double best_t = 1e300;
  const double cap = (double)h->cus * 4 * 64 * 3;
  const int widths[] = {64, 128, 256};
  const int segs[] = {8, 16, 32, 64, 128, 256, 512, 0};
  for (int w : widths)
    for (int sg : segs) {
      long long items, lane_iters;
      int longest;
      shape_cost(h->prm, (int)h->esize, w, sg, &items, &lane_iters, &longest);
      const double t = std::max((double)lane_iters / cap, longest / 3.0);
      if (t < best_t * 0.999) {
        best_t = t;
        best = lbm_axi_launch{w, sg, h->n > 1 ? 1 : 0, 0, 1, regf, 1};
      }
    }
  return best;
}

lbm_status upload_items(lbm_axi_s* h, const std::vector<WorkItem>& items) {
  if (items.size() > h->items_cap) {
    if (h->d_items) HIPCHK(hipFree(h->d_items));
    h->d_items = nullptr;
    const size_t cap = std::max<size_t>(items.size(), 1024);
    HIPCHK(hipMalloc(&h->d_items, cap * sizeof(WorkItem)));
    h->items_cap = cap;
  }
  HIPCHK(hipMemcpyAsync(h->d_items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->n_items = (int)items.size();
  return LBM_OK;
}

void drop_graph(lbm_axi_s* h) {
  for (auto& L : h->grp)
    for (auto& x : L.gexec)
      if (x) {
        (void)hipGraphExecDestroy(x);
        x = nullptr;
      }
}

lbm_status apply_launch(lbm_axi_s* h, const lbm_axi_launch& c0) {
  lbm_axi_launch c = c0;
  if (c.streams == 0) c.streams = 1;
  if (!valid_width(c.width)) return LBM_ERR_UNSUPPORTED;
  if (c.seg_rows != 0 && c.seg_rows < 8) return LBM_ERR_ARG;
  if (c.grid < 0 || (c.regf != 0 && c.regf != 1) || c.xcd_swizzle < 0 || c.xcd_swizzle > 2) return LBM_ERR_ARG;
  if (c.streams < 1 || c.streams > kMaxStreams || c.streams > h->n) return LBM_ERR_ARG;
  for (int g = 1; g < c.streams; ++g) {
    if (!h->grp[g].st) HIPCHK(hipStreamCreateWithFlags(&h->grp[g].st, hipStreamNonBlocking));
    if (!h->grp[g].done) HIPCHK(hipEventCreateWithFlags(&h->grp[g].done, hipEventDisableTiming));
  }
  if (c.streams > 1 && !h->fork) HIPCHK(hipEventCreateWithFlags(&h->fork, hipEventDisableTiming));
  int first[kMaxStreams] = {}, count[kMaxStreams] = {};
  lbm_status s = upload_items(h, launch_items(h->prm, (int)h->esize, c, first, count));
  if (s != LBM_OK) return s;
  drop_graph(h);
  h->launch = c;
  h->n_groups = c.streams;
  h->grp[0].st = h->stream;
  for (int g = 0; g < c.streams; ++g) {
    h->grp[g].first = first[g];
    h->grp[g].count = count[g];
  }
  return LBM_OK;
}

int grid_of(const lbm_axi_s* h, int n_items) {
  if (!h->launch.persistent) return n_items;
  int g = h->launch.grid > 0 ? h->launch.grid : h->cus * (h->launch.width <= 128 ? 8 : 4);
  return std::max(1, std::min(g, n_items));
}

// One step of group grp from fbuf[cur] into fbuf[cur ^ 1], on the group's stream.
template <typename R>
hipError_t enqueue_sweep(lbm_axi_s* h, int grp, int cur) {
  const auto& L = h->grp[grp];
  SweepArgs<R> g{};
  g.fin = static_cast<const R*>(h->fbuf[cur]);
  g.fout = static_cast<R*>(h->fbuf[cur ^ 1]);
  g.inst = h->d_inst;
  g.items = h->d_items + L.first;
  g.n_items = L.count;
  g.xcd_swizzle = h->launch.xcd_swizzle == 1;
  g.queue = h->d_queue + 2 * grp;
  g.err = h->d_err;
  return sweep_dispatch<R>(g, h->launch.width, false, h->launch.persistent != 0, h->launch.regf != 0, h->any_guo,
                           h->any_mid, grid_of(h, L.count), L.st);
}

lbm_status group_steps_eager(lbm_axi_s* h, int grp, int cur, int64_t nsteps) {
  for (int64_t s = 0; s < nsteps; ++s, cur ^= 1) {
    hipError_t e = h->prec == LBM_PREC_FP32 ? enqueue_sweep<float>(h, grp, cur) : enqueue_sweep<double>(h, grp, cur);
    if (e != hipSuccess) return LBM_ERR_HIP;
  }
  return LBM_OK;
}

lbm_status capture_group(lbm_axi_s* h, int grp, int cur) {
  auto& L = h->grp[grp];
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(L.st, hipStreamCaptureModeThreadLocal));
  lbm_status s = group_steps_eager(h, grp, cur, h->graph_chunk);
  hipError_t ee = hipStreamEndCapture(L.st, &graph);
  if (s != LBM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (ee != hipSuccess) return LBM_ERR_HIP;
  hipError_t ie = hipGraphInstantiate(&L.gexec[cur], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    L.gexec[cur] = nullptr;
    return LBM_ERR_HIP;
  }
  // the executable's one-time device set-up now, not in its first launch
  HIPCHK(hipGraphUpload(L.gexec[cur], L.st));
  return LBM_OK;
}

// nsteps steps of every instance, ordered after earlier work on the handle's stream and
// before later work on it.  Whole graph chunks are replayed (a chunk is even, so it ends on
// the buffer it started from; lbm_axi_set_graph_chunk captures the chunks of both starting
// buffers, and one dropped by a change of launch shape is captured again here when
// needed), the rest launched one by one; both go out one step or chunk per group in turn,
// so that every group's stream has work from the start.
lbm_status run_steps(lbm_axi_s* h, int64_t nsteps, bool graphs) {
  if (nsteps == 0) return LBM_OK;
  const int cur = h->cur;
  if (h->n_groups > 1) {
    HIPCHK(hipEventRecord(h->fork, h->stream));
    for (int g = 1; g < h->n_groups; ++g) HIPCHK(hipStreamWaitEvent(h->grp[g].st, h->fork, 0));
  }
  lbm_status st = LBM_OK;
  int64_t left = nsteps;
  if (graphs && h->graph_chunk > 0 && left >= h->graph_chunk) {
    for (int g = 0; g < h->n_groups && st == LBM_OK; ++g)
      if (!h->grp[g].gexec[cur]) st = capture_group(h, g, cur);
    for (; left >= h->graph_chunk && st == LBM_OK; left -= h->graph_chunk)
      for (int g = 0; g < h->n_groups && st == LBM_OK; ++g)
        if (hipGraphLaunch(h->grp[g].gexec[cur], h->grp[g].st) != hipSuccess) st = LBM_ERR_HIP;
  }
  for (int64_t s = 0; s < left && st == LBM_OK; ++s)
    for (int g = 0; g < h->n_groups && st == LBM_OK; ++g) {
      const int c = cur ^ (int)(s & 1);
      if ((h->prec == LBM_PREC_FP32 ? enqueue_sweep<float>(h, g, c) : enqueue_sweep<double>(h, g, c)) != hipSuccess)
        st = LBM_ERR_HIP;
    }
  for (int g = 1; g < h->n_groups; ++g)  // join, also after a failure
    if (hipEventRecord(h->grp[g].done, h->grp[g].st) != hipSuccess ||
        hipStreamWaitEvent(h->stream, h->grp[g].done, 0) != hipSuccess)
      st = LBM_ERR_HIP;
  if (st == LBM_OK) h->cur = cur ^ (int)(nsteps & 1);
  return st;
}

lbm_status enqueue_steps_eager(lbm_axi_s* h, int64_t nsteps) { return run_steps(h, nsteps, false); }
lbm_status enqueue_steps(lbm_axi_s* h, int64_t nsteps) { return run_steps(h, nsteps, true); }

// The sticky device error bits of the handle (k < 0: any instance) or of instance k.
lbm_status read_err(lbm_axi_s* h, int k = -1) {
  int e = 0;
  HIPCHK(hipMemcpyAsync(&e, h->d_err + (k < 0 ? 0 : 1 + k), sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (e & 2) return LBM_ERR_NONFINITE;
  if (e & 1) return LBM_ERR_EOS_DOMAIN;
  return LBM_OK;
}

// The step kernel addresses the rows of a work item with 32-bit byte offsets from one
// descriptor: a segment of at least 8 rows must fit (only rows of many megabytes fail).
bool offsets_fit(const lbm_axi_params& p, int esize) { return max_item_rows(row_pitch(p.nz, esize), esize) >= 8; }

size_t f_bytes_of(int n, const lbm_axi_params* params, int prec, long long* felems_out,
                  std::vector<long long>* bases) {
  long long off = 0;
  const int esize = prec == LBM_PREC_FP32 ? 4 : 8;
  for (int k = 0; k < n; ++k) {
    if (bases) bases->push_back(off);
    const long long nn = 9LL * row_pitch(params[k].nz, esize) * params[k].nr;
    off += (nn + 63) / 64 * 64;  // every instance starts on a 256-byte boundary
  }
  if (felems_out) *felems_out = off;
  return (size_t)off * esize;
}

void free_all(lbm_axi_s* h) {
  drop_graph(h);
  if (h->own_f) {
    if (h->fbuf[0]) (void)hipFree(h->fbuf[0]);
  }
  void* ptrs[] = {h->d_inst, h->d_items, h->d_queue, h->d_err, h->d_rows, h->d_row_start,
                  h->d_part, h->d_out, h->d_geo, h->d_mom, h->d_mitems};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  for (int g = 1; g < kMaxStreams; ++g) {
    if (h->grp[g].st) (void)hipStreamSynchronize(h->grp[g].st);
    if (h->grp[g].st) (void)hipStreamDestroy(h->grp[g].st);
    if (h->grp[g].done) (void)hipEventDestroy(h->grp[g].done);
  }
  if (h->fork) (void)hipEventDestroy(h->fork);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

template <typename R>
hipError_t unstream_into(lbm_axi_s* h, int k, const double* rho0, const double* uz0, const double* ur0,
                         const double* f0) {
  const auto& p = h->prm[k];
  R* dst = static_cast<R*>(h->fbuf[h->cur]) + h->base[k];
  return launch_unstream<R>(dst, p.nz, h->hinst[k].pitch, p.nr, p.bc_top, h->hinst[k].rho_ref, rho0, uz0, ur0, f0,
                            h->stream);
}

// Upload host fields of instance k into a temporary device buffer and build its populations.
lbm_status load_instance(lbm_axi_s* h, int k, const double* rho0, const double* uz0, const double* ur0,
                         const double* f0) {
  const auto& p = h->prm[k];
  const size_t n = (size_t)p.nz * p.nr;
  const size_t count = f0 ? 9 * n : 3 * n;
  double* tmp = nullptr;
  HIPCHK(hipMalloc(&tmp, count * sizeof(double)));
  lbm_status st = LBM_OK;
  do {
    double *d_rho = nullptr, *d_uz = nullptr, *d_ur = nullptr, *d_f = nullptr;
    if (f0) {
      d_f = tmp;
      if (hipMemcpyAsync(d_f, f0, 9 * n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess) {
        st = LBM_ERR_HIP;
        break;
      }
    } else {
      d_rho = tmp;
      if (hipMemcpyAsync(d_rho, rho0, n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess) {
        st = LBM_ERR_HIP;
        break;
      }
      if (uz0) {
        d_uz = tmp + n;
        if (hipMemcpyAsync(d_uz, uz0, n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess) {
          st = LBM_ERR_HIP;
          break;
        }
      }
      if (ur0) {
        d_ur = tmp + 2 * n;
        if (hipMemcpyAsync(d_ur, ur0, n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess) {
          st = LBM_ERR_HIP;
          break;
        }
      }
    }
    hipError_t e = h->prec == LBM_PREC_FP32 ? unstream_into<float>(h, k, d_rho, d_uz, d_ur, d_f)
                                            : unstream_into<double>(h, k, d_rho, d_uz, d_ur, d_f);
    if (e != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) st = LBM_ERR_HIP;
  } while (0);
  (void)hipFree(tmp);
  return st;
}

lbm_status create(int n, const lbm_axi_params* params, int prec, const double* const* rho0, void* stream,
                  void* workspace, size_t ws_bytes, lbm_axi_t* out) {
  if (!out || n < 1 || !params) return LBM_ERR_ARG;
  *out = nullptr;
  if (prec != LBM_PREC_FP64 && prec != LBM_PREC_FP32) return LBM_ERR_ARG;
  for (int k = 0; k < n; ++k) {
    lbm_status s = check_params(params[k]);
    if (s != LBM_OK) return s;
  }
  lbm_axi_s* h = new (std::nothrow) lbm_axi_s();
  if (!h) return LBM_ERR_ALLOC;
  h->n = n;
  h->prec = prec;
  h->esize = prec == LBM_PREC_FP32 ? 4 : 8;
  h->prm.assign(params, params + n);
  const size_t fb = f_bytes_of(n, params, prec, &h->felems, &h->base);
  for (int k = 0; k < n; ++k)
    if (!offsets_fit(params[k], (int)h->esize)) {
      delete h;
      return LBM_ERR_UNSUPPORTED;
    }
  for (int k = 0; k < n; ++k) {
    const double rref = prec == LBM_PREC_FP32 ? reference_density(params[k], rho0[k]) : 0.0;
    h->hinst.push_back(make_inst(params[k], h->base[k], rref, h->esize));
    h->nodes += (long long)params[k].nz * params[k].nr;
    h->any_guo = h->any_guo || params[k].forcing == LBM_FORCING_GUO;
    h->any_mid = h->any_mid || (params[k].source_mid != 0 && params[k].axisym != 0);
  }
  lbm_status st = LBM_OK;
  auto fail = [&](lbm_status s) {
    free_all(h);
    delete h;
    return s;
  };
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(LBM_ERR_HIP);
  h->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  h->device = dev;
  // the static scratch of lbm_axi_mass_async on this device (looked up once per device; a
  // failure only disables that entry point, which then reports it)
  (void)scratch_attach();
  if (stream) {
    h->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return fail(LBM_ERR_HIP);
    h->own_stream = true;
  }
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess)
    return fail(LBM_ERR_HIP);
  if (workspace) {
    if (ws_bytes < 2 * fb || (reinterpret_cast<uintptr_t>(workspace) & 255)) return fail(LBM_ERR_ALLOC);
    h->fbuf[0] = workspace;
    h->own_f = false;
  } else {
    if (hipMalloc(&h->fbuf[0], 2 * fb) != hipSuccess) return fail(LBM_ERR_ALLOC);
    h->own_f = true;
  }
  h->fbuf[1] = static_cast<char*>(h->fbuf[0]) + fb;
  // rows of every instance, for the reductions
  std::vector<RowRef> rows;
  std::vector<int> row_start;
  for (int k = 0; k < n; ++k) {
    row_start.push_back((int)rows.size());
    for (int j = 0; j < params[k].nr; ++j) rows.push_back(RowRef{k, j});
  }
  row_start.push_back((int)rows.size());
  h->n_rows = (int)rows.size();
  if (hipMalloc(&h->d_inst, n * sizeof(InstDev)) != hipSuccess ||
      hipMalloc(&h->d_queue, 2 * kMaxStreams * sizeof(int)) != hipSuccess ||
      hipMalloc(&h->d_err, (n + 1) * sizeof(int)) != hipSuccess ||
      hipMalloc(&h->d_rows, rows.size() * sizeof(RowRef)) != hipSuccess ||
      hipMalloc(&h->d_row_start, row_start.size() * sizeof(int)) != hipSuccess ||
      hipMalloc(&h->d_part, rows.size() * 4 * sizeof(double)) != hipSuccess ||
      hipMalloc(&h->d_out, n * sizeof(double)) != hipSuccess ||
      hipMalloc(&h->d_geo, 3 * n * sizeof(double)) != hipSuccess)
    return fail(LBM_ERR_ALLOC);
  if (hipMemcpy(h->d_inst, h->hinst.data(), n * sizeof(InstDev), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_rows, rows.data(), rows.size() * sizeof(RowRef), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_row_start, row_start.data(), row_start.size() * sizeof(int), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemset(h->d_queue, 0, 2 * kMaxStreams * sizeof(int)) != hipSuccess ||
      hipMemset(h->d_err, 0, (n + 1) * sizeof(int)) != hipSuccess)
    return fail(LBM_ERR_HIP);
  st = apply_launch(h, default_launch(h));
  if (st != LBM_OK) return fail(st);
  *out = h;
  return LBM_OK;
}

// The moments launch of instance k (its own work list, one workgroup per item).
template <typename R>
hipError_t enqueue_moments(lbm_axi_s* h, int k, double* mr, double* mz, double* mu) {
  SweepArgs<R> g{};
  g.fin = static_cast<const R*>(h->fbuf[h->cur]);
  g.fout = static_cast<R*>(h->fbuf[h->cur ^ 1]);
  g.inst = h->d_inst;
  g.items = h->d_mitems + h->mfirst[k];
  g.n_items = h->mcount[k];
  g.xcd_swizzle = 0;
  g.queue = h->d_queue;
  g.err = h->d_err;
  g.mrho = mr;
  g.muz = mz;
  g.mur = mu;
  return sweep_dispatch<R>(g, h->launch.width, true, false, false, false, false, g.n_items, h->stream);
}

// Work lists of the moments launches and the field buffer, (re)built when first needed and
// when the strip width or segment length has changed since.
lbm_status prepare_moments(lbm_axi_s* h) {
  if (!h->d_mom) {
    size_t most = 0;
    for (const auto& p : h->prm) most = std::max(most, (size_t)p.nz * p.nr);
    HIPCHK(hipMalloc(&h->d_mom, 3 * most * sizeof(double)));
  }
  if (h->m_width == h->launch.width && h->m_seg == h->launch.seg_rows) return LBM_OK;
  std::vector<WorkItem> all;
  h->mfirst.assign(h->n, 0);
  h->mcount.assign(h->n, 0);
  for (int k = 0; k < h->n; ++k) {
    std::vector<char> only(h->n, 0);
    only[k] = 1;
    const std::vector<WorkItem> items = build_items(
        h->prm, (int)h->esize, lbm_axi_launch{h->launch.width, h->launch.seg_rows, 0, 0, 0, 0, 1}, only);
    h->mfirst[k] = (int)all.size();
    h->mcount[k] = (int)items.size();
    all.insert(all.end(), items.begin(), items.end());
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  if (h->d_mitems) HIPCHK(hipFree(h->d_mitems));
  h->d_mitems = nullptr;
  h->m_width = 0;
  HIPCHK(hipMalloc(&h->d_mitems, all.size() * sizeof(WorkItem)));
  HIPCHK(hipMemcpy(h->d_mitems, all.data(), all.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  h->m_width = h->launch.width;
  h->m_seg = h->launch.seg_rows;
  return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_axi_status_string(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_ARG: return "invalid argument";
    case LBM_ERR_ALLOC: return "allocation failed or workspace too small";
    case LBM_ERR_HIP: return "HIP runtime error";
    case LBM_ERR_EOS_DOMAIN: return "equation-of-state domain left (rho <= 0 or psi not real)";
    case LBM_ERR_NONFINITE: return "non-finite value";
    case LBM_ERR_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

lbm_status lbm_axi_eos_critical(const lbm_axi_params* p, double* rho_c, double* T_c, double* P_c) {
  if (!p || !rho_c || !T_c || !P_c) return LBM_ERR_ARG;
  return eos_critical(*p, rho_c, T_c, P_c);
}

lbm_status lbm_axi_eos_coexistence(const lbm_axi_params* p, double* rho_v, double* rho_l, double* p_sat) {
  if (!p || !rho_v || !rho_l || !p_sat) return LBM_ERR_ARG;
  return eos_coexistence(*p, rho_v, rho_l, p_sat);
}

lbm_status lbm_axi_workspace_bytes(int32_t n, const lbm_axi_params* params, int32_t precision, size_t* bytes) {
  if (n < 1 || !params || !bytes) return LBM_ERR_ARG;
  if (precision != LBM_PREC_FP64 && precision != LBM_PREC_FP32) return LBM_ERR_ARG;
  for (int k = 0; k < n; ++k) {
    lbm_status s = check_params(params[k]);
    if (s != LBM_OK) return s;
  }
  const size_t fb = f_bytes_of(n, params, precision, nullptr, nullptr);
  for (int k = 0; k < n; ++k)
    if (!offsets_fit(params[k], precision == LBM_PREC_FP32 ? 4 : 8)) return LBM_ERR_UNSUPPORTED;
  *bytes = 2 * fb;
  return LBM_OK;
}

lbm_status lbm_axi_batch_init_ws(int32_t n, const lbm_axi_params* params, int32_t precision,
                                 const double* const* rho0, void* stream, void* workspace,
                                 size_t workspace_bytes, lbm_axi_t* out) {
  if (!rho0 || !params || n < 1 || !out) return LBM_ERR_ARG;
  for (int k = 0; k < n; ++k) {
    if (!rho0[k]) return LBM_ERR_ARG;
    lbm_status s = check_params(params[k]);
    if (s != LBM_OK) return s;
    s = check_rho0(params[k], rho0[k]);
    if (s != LBM_OK) return s;
  }
  lbm_axi_t h = nullptr;
  lbm_status s = create(n, params, precision, rho0, stream, workspace, workspace_bytes, &h);
  if (s != LBM_OK) return s;
  for (int k = 0; k < n && s == LBM_OK; ++k) s = load_instance(h, k, rho0[k], nullptr, nullptr, nullptr);
  if (s != LBM_OK) {
    free_all(h);
    delete h;
    return s;
  }
  *out = h;
  return LBM_OK;
}

lbm_status lbm_axi_batch_init(int32_t n, const lbm_axi_params* params, int32_t precision,
                              const double* const* rho0, void* stream, lbm_axi_t* out) {
  return lbm_axi_batch_init_ws(n, params, precision, rho0, stream, nullptr, 0, out);
}

lbm_status lbm_axi_init(const lbm_axi_params* p, int32_t precision, const double* rho0, const double* uz0,
                        const double* ur0, void* stream, lbm_axi_t* out) {
  if (!p || !rho0 || !out) return LBM_ERR_ARG;
  lbm_status s = check_params(*p);
  if (s != LBM_OK) return s;
  s = check_rho0(*p, rho0);
  if (s != LBM_OK) return s;
  const long long n = (long long)p->nz * p->nr;
  for (const double* u : {uz0, ur0})
    if (u)
      for (long long x = 0; x < n; ++x)
        if (!std::isfinite(u[x])) return LBM_ERR_NONFINITE;
  lbm_axi_t h = nullptr;
  s = create(1, p, precision, &rho0, stream, nullptr, 0, &h);
  if (s != LBM_OK) return s;
  s = load_instance(h, 0, rho0, uz0, ur0, nullptr);
  if (s != LBM_OK) {
    free_all(h);
    delete h;
    return s;
  }
  *out = h;
  return LBM_OK;
}

void lbm_axi_destroy(lbm_axi_t h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  free_all(h);
  delete h;
}

lbm_status lbm_axi_step(lbm_axi_t h, int64_t nsteps) {
  if (!h || nsteps < 0) return LBM_ERR_ARG;
  return enqueue_steps(h, nsteps);
}

lbm_status lbm_axi_step_timed(lbm_axi_t h, int64_t nsteps, double* ms) {
  if (!h || nsteps < 0 || !ms) return LBM_ERR_ARG;
  HIPCHK(hipEventRecord(h->ev0, h->stream));
  lbm_status s = enqueue_steps(h, nsteps);
  if (s != LBM_OK) return s;
  HIPCHK(hipEventRecord(h->ev1, h->stream));
  HIPCHK(hipEventSynchronize(h->ev1));
  float t = 0.f;
  HIPCHK(hipEventElapsedTime(&t, h->ev0, h->ev1));
  *ms = t;
  return read_err(h);
}

lbm_status lbm_axi_sync(lbm_axi_t h) {
  if (!h) return LBM_ERR_ARG;
  return read_err(h);
}

lbm_status lbm_axi_errors(lbm_axi_t h, int32_t* flags) {
  if (!h || !flags) return LBM_ERR_ARG;
  HIPCHK(hipMemcpyAsync(flags, h->d_err + 1, h->n * sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

lbm_status lbm_axi_set_graph_chunk(lbm_axi_t h, int32_t chunk) {
  if (!h || chunk < 0 || (chunk > 0 && (chunk < 2 || (chunk & 1)))) return LBM_ERR_ARG;
  drop_graph(h);
  h->graph_chunk = chunk;
  // capture now the chunks from both buffers, so that no later step call (one that starts
  // on the other buffer after an odd number of eager steps, say) waits for a capture
  for (int b = 0; b < 2 && chunk > 0; ++b)
    for (int g = 0; g < h->n_groups; ++g) {
      lbm_status s = capture_group(h, g, h->cur ^ b);
      if (s != LBM_OK) return s;
    }
  for (int g = 0; g < h->n_groups && chunk > 0; ++g) HIPCHK(hipStreamSynchronize(h->grp[g].st));
  return LBM_OK;
}

lbm_status lbm_axi_moments(lbm_axi_t h, int32_t k, double* rho, double* uz, double* ur) {
  if (!h || k < 0 || k >= h->n || !rho || !uz || !ur) return LBM_ERR_ARG;
  const auto& p = h->prm[k];
  const size_t n = (size_t)p.nz * p.nr;
  lbm_status st = prepare_moments(h);
  if (st != LBM_OK) return st;
  double* tmp = h->d_mom;
  hipError_t e = h->prec == LBM_PREC_FP32 ? enqueue_moments<float>(h, k, tmp, tmp + n, tmp + 2 * n)
                                          : enqueue_moments<double>(h, k, tmp, tmp + n, tmp + 2 * n);
  if (e != hipSuccess ||
      hipMemcpyAsync(rho, tmp, n * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipMemcpyAsync(uz, tmp + n, n * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipMemcpyAsync(ur, tmp + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return LBM_ERR_HIP;
  return read_err(h, k);
}

static lbm_status reduce(lbm_axi_t h, int K, double* out) {
  hipError_t e = h->prec == LBM_PREC_FP32
                     ? launch_rows<float>(K, static_cast<const float*>(h->fbuf[h->cur]), h->d_inst, h->d_rows,
                                          h->n_rows, h->d_geo, h->d_part, h->stream)
                     : launch_rows<double>(K, static_cast<const double*>(h->fbuf[h->cur]), h->d_inst, h->d_rows,
                                           h->n_rows, h->d_geo, h->d_part, h->stream);
  if (e != hipSuccess) return LBM_ERR_HIP;
  HIPCHK(launch_finish(K, h->d_part, h->d_row_start, h->d_inst, h->n, h->d_out, h->stream));
  HIPCHK(hipMemcpyAsync(out, h->d_out, h->n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return read_err(h);
}

lbm_status lbm_axi_mass(lbm_axi_t h, double* mass) {
  if (!h || !mass) return LBM_ERR_ARG;
  return reduce(h, 1, mass);
}

lbm_status lbm_axi_mass_async(lbm_axi_t h, double* mass_dev) {
  if (!h || !mass_dev) return LBM_ERR_ARG;
  // one FP64 partial per row of every instance in the device's static scratch
  if ((size_t)h->n_rows * sizeof(double) > scratch_bytes()) return LBM_ERR_UNSUPPORTED;
  double* part = static_cast<double*>(scratch_ptr(h->device));
  if (!part) return LBM_ERR_HIP;
  hipError_t e = h->prec == LBM_PREC_FP32
                     ? launch_rows<float>(1, static_cast<const float*>(h->fbuf[h->cur]), h->d_inst, h->d_rows,
                                          h->n_rows, nullptr, part, h->stream)
                     : launch_rows<double>(1, static_cast<const double*>(h->fbuf[h->cur]), h->d_inst, h->d_rows,
                                           h->n_rows, nullptr, part, h->stream);
  if (e != hipSuccess) return LBM_ERR_HIP;
  HIPCHK(launch_finish(1, part, h->d_row_start, h->d_inst, h->n, mass_dev, h->stream));
  return LBM_OK;
}

lbm_status lbm_axi_laplace(lbm_axi_t h, const double* zc, const double* r_in, const double* r_out, double* dp) {
  if (!h || !zc || !r_in || !r_out || !dp) return LBM_ERR_ARG;
  std::vector<double> geo(3 * h->n);
  for (int k = 0; k < h->n; ++k) {
    geo[3 * k] = zc[k];
    geo[3 * k + 1] = r_in[k];
    geo[3 * k + 2] = r_out[k];
  }
  HIPCHK(hipMemcpyAsync(h->d_geo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
  return reduce(h, 4, dp);
}

lbm_status lbm_axi_axis_interface(lbm_axi_t h, const double* zc, const double* thr, double* z) {
  if (!h || !zc || !thr || !z) return LBM_ERR_ARG;
  std::vector<double> geo(2 * h->n);
  for (int k = 0; k < h->n; ++k) {
    if (!(zc[k] >= 0.0) || !(zc[k] < h->prm[k].nz) || !std::isfinite(thr[k])) return LBM_ERR_ARG;
    geo[2 * k] = zc[k];
    geo[2 * k + 1] = thr[k];
  }
  HIPCHK(hipMemcpyAsync(h->d_geo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
  const hipError_t e =
      h->prec == LBM_PREC_FP32
          ? launch_axis<float>(static_cast<const float*>(h->fbuf[h->cur]), h->d_inst, h->n, h->d_geo, h->d_out,
                               h->stream)
          : launch_axis<double>(static_cast<const double*>(h->fbuf[h->cur]), h->d_inst, h->n, h->d_geo, h->d_out,
                                h->stream);
  if (e != hipSuccess) return LBM_ERR_HIP;
  HIPCHK(hipMemcpyAsync(z, h->d_out, h->n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return read_err(h);
}

lbm_status lbm_axi_get_f(lbm_axi_t h, int32_t k, double* f) {
  if (!h || k < 0 || k >= h->n || !f) return LBM_ERR_ARG;
  const auto& p = h->prm[k];
  const size_t n = (size_t)p.nz * p.nr;
  double* tmp = nullptr;
  HIPCHK(hipMalloc(&tmp, 9 * n * sizeof(double)));
  hipError_t e =
      h->prec == LBM_PREC_FP32
          ? launch_export<float>(static_cast<const float*>(h->fbuf[h->cur]) + h->base[k], p.nz, h->hinst[k].pitch,
                                 p.nr, p.bc_top, h->hinst[k].rho_ref, tmp, h->stream)
          : launch_export<double>(static_cast<const double*>(h->fbuf[h->cur]) + h->base[k], p.nz,
                                  h->hinst[k].pitch, p.nr, p.bc_top, h->hinst[k].rho_ref, tmp, h->stream);
  lbm_status st = LBM_OK;
  if (e != hipSuccess ||
      hipMemcpyAsync(f, tmp, 9 * n * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    st = LBM_ERR_HIP;
  (void)hipFree(tmp);
  if (st != LBM_OK) return st;
  return read_err(h, k);
}

lbm_status lbm_axi_set_f(lbm_axi_t h, int32_t k, const double* f) {
  if (!h || k < 0 || k >= h->n || !f) return LBM_ERR_ARG;
  const auto& p = h->prm[k];
  const size_t n = (size_t)p.nz * p.nr;
  for (size_t x = 0; x < 9 * n; ++x)
    if (!std::isfinite(f[x])) return LBM_ERR_NONFINITE;
  HIPCHK(hipStreamSynchronize(h->stream));
  return load_instance(h, k, nullptr, nullptr, nullptr, f);
}

lbm_status lbm_axi_get_launch(lbm_axi_t h, lbm_axi_launch* cfg) {
  if (!h || !cfg) return LBM_ERR_ARG;
  *cfg = h->launch;
  return LBM_OK;
}

lbm_status lbm_axi_set_launch(lbm_axi_t h, const lbm_axi_launch* cfg) {
  if (!h || !cfg) return LBM_ERR_ARG;
  HIPCHK(hipStreamSynchronize(h->stream));
  return apply_launch(h, *cfg);
}

lbm_status lbm_axi_sizes(lbm_axi_t h, int32_t* n, int64_t* nodes, int64_t* f_bytes) {
  if (!h) return LBM_ERR_ARG;
  if (n) *n = h->n;
  if (nodes) *nodes = h->nodes;
  if (f_bytes) *f_bytes = (int64_t)(h->felems * (long long)h->esize);
  return LBM_OK;
}

lbm_status lbm_axi_stream_copy(int64_t bytes, int32_t iters, double* gbps) {
  if (bytes < 16 || (bytes & 15) || iters < 1 || !gbps) return LBM_ERR_ARG;
  void *a = nullptr, *b = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  lbm_status st = LBM_OK;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) st = LBM_ERR_ALLOC;
  if (st == LBM_OK && (hipMemset(a, 0, bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
                       hipEventCreate(&e1) != hipSuccess))
    st = LBM_ERR_HIP;
  if (st == LBM_OK && launch_copy(a, b, bytes, nullptr) != hipSuccess) st = LBM_ERR_HIP;  // warm-up
  if (st == LBM_OK) {
    (void)hipEventRecord(e0, nullptr);
    for (int i = 0; i < iters && st == LBM_OK; ++i)
      if (launch_copy(a, b, bytes, nullptr) != hipSuccess) st = LBM_ERR_HIP;
    (void)hipEventRecord(e1, nullptr);
    float ms = 0.f;
    if (st == LBM_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = LBM_ERR_HIP;
    if (st == LBM_OK) *gbps = 2.0 * (double)bytes * iters / (ms * 1e-3) / 1e9;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  return st;
}

lbm_status lbm_axi_autotune(lbm_axi_t h, int32_t steps_per_trial, lbm_axi_launch* best, double* best_ms) {
  if (!h || steps_per_trial < 1) return LBM_ERR_ARG;
  HIPCHK(hipStreamSynchronize(h->stream));
  // A state that has already left the EOS domain (or gone non-finite) is reported, not tuned:
  // its sticky error words stay as they are.
  std::vector<int> err_words(h->n + 1, 0);
  HIPCHK(hipMemcpy(err_words.data(), h->d_err, err_words.size() * sizeof(int), hipMemcpyDeviceToHost));
  if (err_words[0] & 2) return LBM_ERR_NONFINITE;
  if (err_words[0] & 1) return LBM_ERR_EOS_DOMAIN;
  const size_t fb = (size_t)h->felems * h->esize;
  void* save = nullptr;
  HIPCHK(hipMalloc(&save, fb));
  const int cur0 = h->cur;
  lbm_status st = LBM_OK;
  if (hipMemcpyAsync(save, h->fbuf[cur0], fb, hipMemcpyDeviceToDevice, h->stream) != hipSuccess) st = LBM_ERR_HIP;
  const lbm_axi_launch keep = h->launch;
  const int keep_chunk = h->graph_chunk;
  h->graph_chunk = 0;
  // Time one candidate for `steps` steps after a warm-up step, then restore the state.
  auto trial = [&](const lbm_axi_launch& c, int steps, double* ms) -> lbm_status {
    lbm_status s = apply_launch(h, c);
    if (s != LBM_OK) return s;
    if (enqueue_steps_eager(h, 1) != LBM_OK) return LBM_ERR_HIP;
    float t = 0.f;
    if (hipEventRecord(h->ev0, h->stream) != hipSuccess || enqueue_steps_eager(h, steps) != LBM_OK ||
        hipEventRecord(h->ev1, h->stream) != hipSuccess || hipEventSynchronize(h->ev1) != hipSuccess ||
        hipEventElapsedTime(&t, h->ev0, h->ev1) != hipSuccess)
      return LBM_ERR_HIP;
    *ms = t / steps;
    h->cur = cur0;
    if (hipMemcpyAsync(h->fbuf[cur0], save, fb, hipMemcpyDeviceToDevice, h->stream) != hipSuccess) return LBM_ERR_HIP;
    return LBM_OK;
  };
  // Pass 1: every candidate, steps_per_trial steps.  Pass 2: the four fastest again, twice,
  // each time with four times the steps and at least ~20 ms of them, so that run-to-run
  // noise does not pick the winner.
  std::vector<std::pair<double, lbm_axi_launch>> timed;
  int maxnz = 0;
  for (auto& p : h->prm) maxnz = std::max(maxnz, p.nz);
  const int widths[] = {64, 128, 256};
  const int segs[] = {32, 40, 48, 64, 80, 96, 112, 128, 192, 256, 512, 0};
  for (int w : widths) {
    if (w > 64 && maxnz + 12 <= w / 2) continue;  // most lanes would duplicate columns
    for (int sg : segs)
      for (int v = 0; v < 8 && st == LBM_OK; ++v) {
        // v < 4: bit 0 persistent, bit 1 populations in registers (XCD swizzle);
        // v >= 4: one item per workgroup, longest first, bit 0 populations in registers,
        // bit 1 row bands kept on one XCD
        const lbm_axi_launch c = v < 4 ? lbm_axi_launch{w, sg, v & 1, 0, 1, v >> 1, 1}
                                       : lbm_axi_launch{w, sg, 0, 0, v >= 6 ? 2 : 0, v & 1, 1};
        double ms = 0.0;
        const lbm_status s = trial(c, steps_per_trial, &ms);
        if (s == LBM_ERR_HIP) st = s;
        if (s == LBM_OK) timed.push_back({ms, c});
      }
  }
  // Batches: two stream groups, which favour shorter segments than one launch (the tail of
  // one group's step is filled by the other's).  Three groups run about as fast, four slower;
  // one workgroup per item with row bands on one XCD: persistent grids sized for the whole
  // chip, one per group, measured twice as slow.
  const int stream_segs[] = {48, 64, 80, 96, 112};
  for (int nl = 2; nl <= std::min(2, h->n); ++nl)
    for (int w : widths) {
      if (w == 64 || maxnz + 12 <= w / 2) continue;
      for (int sg : stream_segs)
        for (int regf = 0; regf < 2 && st == LBM_OK; ++regf) {
          const lbm_axi_launch c{w, sg, 0, 0, 2, regf, nl};
          double ms = 0.0;
          const lbm_status s = trial(c, steps_per_trial, &ms);
          if (s == LBM_ERR_HIP) st = s;
          if (s == LBM_OK) timed.push_back({ms, c});
        }
    }
  std::sort(timed.begin(), timed.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
  lbm_axi_launch win = keep;
  double win_ms = 1e300;
  for (size_t i = 0; i < timed.size() && i < 4 && st == LBM_OK; ++i) {
    // at least four times the first pass's steps and about 20 ms of steps, best of two
    const int steps2 = (int)std::min(200.0, std::max(4.0 * steps_per_trial, std::ceil(20.0 / timed[i].first)));
    for (int rep = 0; rep < 2 && st == LBM_OK; ++rep) {
      double ms = 0.0;
      st = trial(timed[i].second, steps2, &ms);
      if (st == LBM_OK && ms < win_ms) {
        win_ms = ms;
        win = timed[i].second;
      }
    }
  }
  (void)hipStreamSynchronize(h->stream);
  (void)hipFree(save);
  h->graph_chunk = keep_chunk;
  lbm_status s2 = apply_launch(h, st == LBM_OK ? win : keep);
  // The trials stepped copies of the state, which may have raised error bits that the
  // restored state does not have: put back the words read before tuning (all clear).
  if (hipMemcpy(h->d_err, err_words.data(), err_words.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess &&
      st == LBM_OK)
    st = LBM_ERR_HIP;
  if (st != LBM_OK) return st;
  if (s2 != LBM_OK) return s2;
  if (best) *best = h->launch;  // as applied (streams = 0 read as 1)
  if (best_ms) *best_ms = win_ms;
  return LBM_OK;
}

}  // extern "C"
