// Solver handle, SETUP pipeline, SOLVE orchestration and the C-ABI of cpc.h.
//
// SETUP (Section 3.2): validate, ILU(0) on the host, then per level: classical
// C/F splitting and interpolation on the host, Galerkin product R (A P) on the GPU,
// download of the coarse matrix for the next splitting. The coarsest matrix is
// inverted densely (FP64). Sweep schedules and device copies follow.
//
// SOLVE: PCG with all scalars on the device; each iteration is one fixed sequence
// of kernels (optionally replayed from a captured HIP graph); the host reads the
// convergence state after every `check_every` iterations, or, by default, after as
// many as the residual history predicts, and kernels after convergence return
// immediately, so the iteration count is exact.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <thread>
#include <map>
#include <set>
#include <chrono>
#include <exception>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/cpc.h"
#include "host_setup.hpp"
#include "kernels.hpp"
#include "solve_scratch.hpp"

namespace {

thread_local std::string g_last_error;

cpc_status set_err(cpc_status st, const std::string& m) {
  g_last_error = m;
  return st;
}

struct HipError {
  hipError_t e;
  std::string where;
};

#define HIPCHK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) throw HipError{e_, std::string(#expr)};             \
  } while (0)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <typename T>
T* dalloc(size_t count, std::vector<void*>& owned) {
  void* p = nullptr;
  if (count == 0) count = 1;
  HIPCHK(hipMalloc(&p, count * sizeof(T)));
  owned.push_back(p);
  return static_cast<T*>(p);
}

template <typename T, typename A>
T* dupload(const std::vector<T, A>& h, std::vector<void*>& owned, hipStream_t s) {
  T* d = dalloc<T>(h.size(), owned);
  if (!h.empty()) HIPCHK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return d;
}

int pick_tpr(double avg_row) {
  int t = 1;
  while (t < 64 && t * 3 < avg_row) t <<= 1;
  return t;
}

// Entries per lane taken at once by a row product of a small launch: the average a lane
// holds, rounded up to 1, 2 or 4.
int pick_steps(double avg_row, int tpr) {
  const double per_lane = avg_row / tpr;
  return per_lane <= 1.0 ? 1 : (per_lane <= 2.0 ? 2 : 4);
}

}  // namespace

namespace cpc {

struct DevCsr {
  int n = 0, ncols = 0;
  int64_t nnz = 0;
  int* rp = nullptr;
  int* ci = nullptr;
  double* v = nullptr;
  float* v32 = nullptr;
  int* dpos = nullptr;
  int tpr = 1;
  int steps = 1;
  MatDev mat(bool fp32) const {
    MatDev m;
    m.n = n;
    m.rp = rp;
    m.ci = ci;
    m.dpos = dpos;
    m.v = fp32 ? (const void*)v32 : (const void*)v;
    m.fp32 = fp32;
    m.steps = steps;
    return m;
  }
};

// Block substitution with explicit inverses of the diagonal blocks of D+L. Blocks never
// span two systems of a batch: step k of the forward solve takes the k-th block of every
// system at once, step t of the backward solve the t-th block from each system's end
// (one system: one block per step).
struct BlockDense {
  int B = 0;
  std::vector<int> start, rows;    // per block, in forward-step order: first row, rows
  std::vector<long> moff;          // per block: element offset of its inverse
  std::vector<int> fstep;          // forward step k: blocks [fstep[k], fstep[k+1])
  std::vector<int> bblk, bstep;    // backward step t: blocks bblk[bstep[t] .. bstep[t+1])
  std::vector<int> fitem, bitem;   // offsets of each step's row items in the two item lists
  std::vector<int> frow, brow;     // offsets of each step's rows in Loff / Uoff
  const int4* items_f = nullptr;   // row items of the forward steps (device)
  const int4* items_b = nullptr;   // row items of the backward steps (device)
  DenseTriDev dt{};                // the blocks as systems: n, moff, voff per block; M, MT
  DevCsr Loff, Uoff;               // entries left / right of the row's block, rows in step order
  const int* Lrid = nullptr;       // level row of each row of Loff / Uoff (device)
  const int* Urid = nullptr;
  double entries = 0.0;            // stored inverse entries (byte model)
  double stored_bytes = 0.0;       // device bytes of the inverses and their transposes
  std::vector<void*> owned;
  int nblk() const { return (int)start.size(); }
};

struct DevSweepSched {
  SweepDev d{};
  int global_depth = 0;
};

struct Level {
  HostCsr A_host;
  HostCsr P_host;  // prolongation from level+1 to this level
  std::vector<int> cf;
  DevCsr A, P, R;
  DevSweepSched lower, upper;
  SweepPackDev fgs{}, bgs{};  // (D+L) and (D+U) solves of the smoothed rows
  DevCsr Ls;                  // strict lower triangle of the smoothed rows
  int nS = 0;                 // leading rows that are smoothed (systems not at their coarsest level)
  int64_t nnzS = 0;           // nonzeros of those rows
  DenseListDev dense{};       // systems whose coarsest level is this one (exact solve)
  std::vector<int> dense_n;   // their sizes (host)
  void* f = nullptr;  // level vectors (coarse levels), element type = preconditioner precision
  void* u = nullptr;
  void* r = nullptr;
  void* t = nullptr;  // right-hand side of the backward sweep
  // explicit inverses of D+L of the smoothed systems, where they are faster than sweeps
  DenseTriDev dtri{};
  double dense_bytes = 0.0;  // device bytes of those inverses (and transposes)
  void* dense_M = nullptr;     // held here until the setup tuner keeps or drops it
  void* dense_MT = nullptr;    // its transpose (small systems), same ownership
  std::vector<void*> dense_owned;  // the kept inverse (and transpose)
  bool dense_smooth = false;   // smooth through dtri instead of the level-scheduled sweeps
  double dense_entries = 0.0;  // stored lower-triangle entries (byte model)
  // device memory of this level's sweep schedules and packs (replaced by the tuner)
  std::vector<void*> sweep_owned;
  int sweep_rows = 0;  // rows the sweeps cover (all rows at depth 0 for ILU(0), else the smoothed ones)
  int sweep_R = 0;     // rows per block requested for them
  std::vector<int> parts;  // row ranges of the systems among the swept rows (batches; empty: one)
  std::vector<int> part_sys;  // batch system of each part (batches only)
  const int* row_sys = nullptr;  // [rows] batch system of each row of the level (batches only)
  int wave_M = 0;      // segments per block of the one-wave form (0: chosen by rule)
  int wave_stride = -1;  // the matrix's dominant coupling distance (-1: not yet measured)
  // block-dense form of the smoother: block forward/backward substitution with explicit
  // inverses of the diagonal blocks of D+L (levels where it beats the sweeps)
  bool bdense = false;
  BlockDense bd;
};

}  // namespace cpc

constexpr int kNumPrec = CPC_PREC_BBAR + 1;  // preconditioners cpc_solve can run

struct cpc_solver {
  cpc_options opt{};
  // batched solves: the per-system stop flags the preconditioner's kernels skip stopped
  // systems by (set while a batched solve enqueues its work; null otherwise)
  const int* mask_done = nullptr;
  int device = 0;  // the GPU the handle was set up on (current device at setup)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int n = 0;
  int64_t nnz = 0;
  bool f32 = false;  // preconditioner precision
  std::vector<cpc::Level> lev;
  std::vector<double> lu_host;
  double setup_t0 = 0.0;  // wall clock at the start of setup (progress lines)
  // ILU(k) with k > 0 (options.ilu_fill): its own factor, sweep schedules and packs
  bool iluk = false;
  cpc::HostCsr iluF;
  std::vector<int> iluF_lev;
  cpc::DevSweepSched ilu_lower, ilu_upper;
  double ilu_lnnz = 0.0, ilu_unnz = 0.0;  // entries of the applied factor below / on and above the diagonal
  double* lu = nullptr;
  float* lu32 = nullptr;
  cpc::SweepPackDev ilu_l{}, ilu_u{};  // ILU(0) L (lower entries of LU) and U (upper entries, diagonal)
  // PCG vectors
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  // preconditioner temporaries on the finest level (precision of the preconditioner)
  void *pin = nullptr, *u1 = nullptr, *u2 = nullptr, *res = nullptr, *y = nullptr, *w = nullptr, *t = nullptr;
  double* z64tmp = nullptr;  // FP64 temporary for the additive form
  cpc::PcgState* st = nullptr;
  double* partials = nullptr;
  cpc::SweepSync sync{};
  long spin_limit = 1L << 22;
  cpc_stats stats{};
  std::vector<void*> owned;
  std::vector<void*>* cur_owned = &owned;  // where sweep schedules and packs are allocated
  // captured iteration graphs, one per preconditioner
  hipGraphExec_t graph[kNumPrec] = {};
  hipGraph_t graph_src[kNumPrec] = {};
  double* graph_x[kNumPrec] = {};  // x bound into each graph
  const double* op_vals = nullptr;  // values PCG multiplies by (null: the setup matrix)
  // batch of independent systems (cpc_setup_batch)
  bool batch = false;
  int nsys = 1;
  std::vector<int> sys_n, sys_off;
  cpc::BatchDev bd{};
  double* btol = nullptr;
  int* bmaxit = nullptr;
  hipGraphExec_t bgraph[kNumPrec] = {};
  hipGraph_t bgraph_src[kNumPrec] = {};
  double* bgraph_x[kNumPrec] = {};

  ~cpc_solver() {
    for (int i = 0; i < kNumPrec; ++i) {
      if (graph[i]) (void)hipGraphExecDestroy(graph[i]);
      if (graph_src[i]) (void)hipGraphDestroy(graph_src[i]);
      if (bgraph[i]) (void)hipGraphExecDestroy(bgraph[i]);
      if (bgraph_src[i]) (void)hipGraphDestroy(bgraph_src[i]);
    }
    for (auto& L : lev) {
      if (L.dense_M) (void)hipFree(L.dense_M);
      if (L.dense_MT) (void)hipFree(L.dense_MT);
      for (void* ptr : L.sweep_owned) (void)hipFree(ptr);
      for (void* ptr : L.bd.owned) (void)hipFree(ptr);
      for (void* ptr : L.dense_owned) (void)hipFree(ptr);
    }
    for (void* ptr : owned) (void)hipFree(ptr);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace cpc {

static void upload_csr(cpc_solver* h, const HostCsr& a, DevCsr& d, bool with_dpos, std::vector<void*>* into = nullptr,
                       bool with_f32 = true, hipStream_t stream = nullptr) {
  std::vector<void*>& own = into ? *into : h->owned;
  const hipStream_t st = stream ? stream : h->stream;
  d.n = a.n;
  d.ncols = a.ncols;
  d.nnz = a.nnz();
  d.rp = dupload(a.rp, own, st);
  d.ci = dupload(a.ci, own, st);
  d.v = dupload(a.v, own, st);
  if (with_dpos) {
    std::vector<int> dp(a.n, -1);
    for (int i = 0; i < a.n; ++i)
      for (int k = a.rp[i]; k < a.rp[i + 1]; ++k)
        if (a.ci[k] == i) dp[i] = k;
    d.dpos = dupload(dp, own, st);
  }
  d.tpr = pick_tpr(a.n ? (double)d.nnz / a.n : 1.0);
  d.steps = pick_steps(a.n ? (double)d.nnz / a.n : 1.0, d.tpr);
  if (h->f32 && with_f32) {
    d.v32 = dalloc<float>((size_t)d.nnz, own);
    launch_to_f32(st, d.nnz, d.v, d.v32);
  }
}

static HostCsr leading_rows(const HostCsr& a, int nrows) {
  HostCsr t;
  t.n = nrows;
  t.ncols = nrows;
  t.rp.assign(a.rp.begin(), a.rp.begin() + nrows + 1);
  t.ci.assign(a.ci.begin(), a.ci.begin() + t.rp[nrows]);
  t.v.assign(a.v.begin(), a.v.begin() + t.rp[nrows]);
  return t;
}

static DenseListDev upload_dense_list(cpc_solver* h, const std::vector<int>& off, const std::vector<int>& nn,
                                      const std::vector<const std::vector<double>*>& invs) {
  DenseListDev dl{};
  if (off.empty()) return dl;
  std::vector<int> blk_entry, blk_row0;
  std::vector<long> inv_off;
  std::vector<double> inv_all;
  for (size_t e = 0; e < off.size(); ++e) {
    inv_off.push_back((long)inv_all.size());
    inv_all.insert(inv_all.end(), invs[e]->begin(), invs[e]->end());
    for (int r = 0; r < nn[e]; r += 4) {
      blk_entry.push_back((int)e);
      blk_row0.push_back(r);
    }
  }
  dl.nblk = (int)blk_entry.size();
  dl.blk_entry = dupload(blk_entry, h->owned, h->stream);
  dl.blk_row0 = dupload(blk_row0, h->owned, h->stream);
  dl.n = dupload(nn, h->owned, h->stream);
  dl.off = dupload(off, h->owned, h->stream);
  dl.inv_off = dupload(inv_off, h->owned, h->stream);
  dl.inv = dupload(inv_all, h->owned, h->stream);
  return dl;
}

// Galerkin product on the GPU: C = X * Y with the canonical order (rap.hip).
static bool gpu_spgemm(cpc_solver* h, const DevCsr& X, const DevCsr& Y, int ncols, HostCsr& C_host, DevCsr& C,
                       std::string* msg, std::vector<void*>& keep, hipStream_t stream = nullptr) {
  const hipStream_t hs = stream ? stream : h->stream;
  const int nrows = X.n;
  std::vector<void*> tmp;
  int* counts = dalloc<int>(nrows, tmp);
  int* ovf = dalloc<int>(1, tmp);
  bool ok = true;
  try {
    HIPCHK(hipMemsetAsync(ovf, 0, sizeof(int), hs));
    launch_spgemm_count(hs, nrows, X.rp, X.ci, Y.rp, Y.ci, counts, ovf);
    HIPCHK(hipGetLastError());
    std::vector<int> hc(nrows);
    int hovf = 0;
    HIPCHK(hipMemcpyAsync(hc.data(), counts, sizeof(int) * nrows, hipMemcpyDeviceToHost, hs));
    HIPCHK(hipMemcpyAsync(&hovf, ovf, sizeof(int), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipStreamSynchronize(hs));
    // rows wider than the LDS table: counted (and later filled) with a dense accumulator
    // slice of ncols entries per workgroup, at most 64 workgroups and 1 GiB
    std::vector<int> wide;
    for (int i = 0; hovf && i < nrows; ++i)
      if (hc[i] < 0) wide.push_back(i);
    int nwg = 0;
    int* wrows = nullptr;
    int* mark = nullptr;
    if (!wide.empty()) {
      nwg = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)wide.size(), 64,
                                                          (int64_t)(1LL << 30) / (12LL * std::max(ncols, 1))}));
      wrows = dupload(wide, tmp, hs);
      mark = dalloc<int>((size_t)nwg * std::max(ncols, 1), tmp);
      HIPCHK(hipMemsetAsync(mark, 0, sizeof(int) * (size_t)nwg * std::max(ncols, 1), hs));
      launch_spgemm_count_wide(hs, (int)wide.size(), wrows, X.rp, X.ci, Y.rp, Y.ci, ncols, mark, nwg, counts);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(hc.data(), counts, sizeof(int) * nrows, hipMemcpyDeviceToHost, hs));
      HIPCHK(hipStreamSynchronize(hs));
    }
    {
      C_host.n = nrows;
      C_host.ncols = ncols;
      C_host.rp.assign(nrows + 1, 0);
      int64_t tot = 0;
      for (int i = 0; i < nrows; ++i) {
        tot += hc[i];
        if (tot > 2147483647LL) {
          ok = false;
          if (msg) *msg = "Galerkin product exceeds 2^31 entries";
          break;
        }
        C_host.rp[i + 1] = (int)tot;
      }
      if (ok) {
        C.n = nrows;
        C.ncols = ncols;
        C.nnz = tot;
        C.rp = dupload(C_host.rp, keep, hs);
        C.ci = dalloc<int>((size_t)tot, keep);
        C.v = dalloc<double>((size_t)tot, keep);
        HIPCHK(hipMemsetAsync(ovf, 0, sizeof(int), hs));
        launch_spgemm_fill(hs, nrows, X.rp, X.ci, X.v, Y.rp, Y.ci, Y.v, C.rp, C.ci, C.v, ovf);
        if (!wide.empty()) {
          double* acc = dalloc<double>((size_t)nwg * std::max(ncols, 1), tmp);
          HIPCHK(hipMemsetAsync(mark, 0, sizeof(int) * (size_t)nwg * std::max(ncols, 1), hs));
          launch_spgemm_fill_wide(hs, (int)wide.size(), wrows, X.rp, X.ci, X.v, Y.rp, Y.ci, Y.v, ncols, mark, acc,
                                  nwg, C.rp, C.ci, C.v, ovf);
        }
        HIPCHK(hipGetLastError());
        C_host.ci.resize(tot);
        C_host.v.resize(tot);
        HIPCHK(hipMemcpyAsync(C_host.ci.data(), C.ci, sizeof(int) * tot, hipMemcpyDeviceToHost, hs));
        HIPCHK(hipMemcpyAsync(C_host.v.data(), C.v, sizeof(double) * tot, hipMemcpyDeviceToHost, hs));
        HIPCHK(hipMemcpyAsync(&hovf, ovf, sizeof(int), hipMemcpyDeviceToHost, hs));
        HIPCHK(hipStreamSynchronize(hs));
        if (hovf) {
          ok = false;
          if (msg) *msg = "Galerkin product table overflow";
        }
      }
    }
  } catch (...) {
    for (void* ptr : tmp) (void)hipFree(ptr);
    throw;
  }
  for (void* ptr : tmp) (void)hipFree(ptr);
  return ok;
}

static void progress(const cpc_solver* h, const std::string& what) {
  if (h->opt.verbose) {
    std::fprintf(stderr, "[cpc setup %7.2f s] %s\n", now_s() - h->setup_t0, what.c_str());
    std::fflush(stderr);
  }
}

static size_t esz_of(const cpc_solver* h) { return h->f32 ? sizeof(float) : sizeof(double); }

static void* valloc(cpc_solver* h, int n) {
  if (h->f32) return dalloc<float>(n, h->owned);
  return dalloc<double>(n, h->owned);
}

static int choose_block_rows(int n) {
  // One workgroup per block. Up to 8192 rows a single block keeps every dependency
  // inside one workgroup; beyond that, blocks of 4096 rows leave LDS room for the
  // products of a level and give larger levels a workgroup per compute unit.
  return n <= sweep_max_rows_per_block() ? n : 4096;
}

// LDS layout of a sweep workgroup: products | solved values | rows | entry offsets |
// per-level ranges (16 bytes a level). Returns the bytes used.
static int sweep_layout(const SweepSchedule& s, int esz, int pcap, SweepDev& sd) {
  auto al = [](int64_t v) { return (int)((v + 15) & ~int64_t(15)); };
  sd.pcap = pcap;
  sd.off_xs = al(8 * (int64_t)pcap);
  sd.off_rows = sd.off_xs + al((int64_t)esz * s.R);
  sd.off_ptr = sd.off_rows + al(4 * (int64_t)s.R);
  sd.off_meta = sd.off_ptr + al(4 * ((int64_t)s.R + 1));
  sd.lds = sd.off_meta + al(16 * (int64_t)s.max_local_levels);
  return sd.lds;
}

// Schedule of one triangular solve of `a` (forward: lower, backward: upper) in blocks
// of at most R rows, uploaded, with levels cut so that their products fit the LDS the
// block's other arrays leave.
// The four-wave kernel's schedule of one direction with R rows per block, its levels
// cut to fit the LDS budget (host only; throws HipError when no cut fits).
struct SweepPlan {
  SweepSchedule s;
  SweepDev sd{};
};
static SweepPlan plan_sweep(const cpc_solver* h, const HostCsr& a, bool forward, int R,
                            const std::vector<int>* parts = nullptr) {
  const int esz = (int)esz_of(h);
  const int budget = sweep_lds_budget();
  const int nt = sweep_threads();
  SweepPlan pl;
  SweepSchedule& s = pl.s;
  SweepDev& sd = pl.sd;
  s = build_sweep(a, forward, R, 0, parts);
  int room = (budget - 16 - sweep_layout(s, esz, 0, sd)) / 8;
  if (room < nt) throw HipError{hipErrorInvalidValue, "sweep block too large for LDS"};
  int64_t cap = s.max_level_entries;
  for (int tries = 0; cap > room; ++tries) {
    // cutting levels adds levels to the level table: leave some slack and retry
    cap = std::max<int64_t>(nt, (int64_t)(0.9 * room));
    s = build_sweep(a, forward, R, cap, parts);
    room = (budget - 16 - sweep_layout(s, esz, 0, sd)) / 8;
    if (room < nt || tries > 6) throw HipError{hipErrorInvalidValue, "sweep levels do not fit LDS"};
  }
  const int pcap = (int)std::max<int64_t>(nt, std::max<int64_t>(cap, s.max_level_entries));
  if (sweep_layout(s, esz, pcap, sd) > budget) throw HipError{hipErrorInvalidValue, "sweep LDS layout over budget"};
  sd.n = s.n;
  sd.R = s.R;
  sd.nblk = s.nblk;
  sd.nlev = (int)s.lvl_ptr.size() - 1;
  sd.maxl = s.max_local_levels;
  sd.grid = std::min(s.nblk, 1024);
  // four waves per block; a one-wave workgroup (no cross-wave barriers) measured
  // slower even where one block covers the matrix, since a level's entries then take
  // four times as many steps per lane
  sd.nt = h->opt.sweep_threads == 64 ? 64 : 256;
  return pl;
}

// parts / part_sys (batches): the system of each block, for the per-system mask (blocks
// then never span two systems).
static void upload_sweep(cpc_solver* h, const SweepPlan& pl, DevSweepSched& d, const std::vector<int>* parts = nullptr,
                         const std::vector<int>* part_sys = nullptr) {
  SweepDev sd = pl.sd;
  if (parts && part_sys && part_sys->size() + 1 == parts->size()) {
    std::vector<int> bs(pl.s.nblk, -1);
    size_t q = 0;
    for (int b = 0; b < pl.s.nblk; ++b) {
      const int r0 = pl.s.blk_row[b], r1 = pl.s.blk_row[b + 1];
      while (q + 1 < parts->size() && (*parts)[q + 1] <= r0) ++q;
      if (q + 1 < parts->size() && r1 <= (*parts)[q + 1]) bs[b] = (*part_sys)[q];
    }
    sd.mask.of = dupload(bs, *h->cur_owned, h->stream);
  }
  sd.blk_row = dupload(pl.s.blk_row, *h->cur_owned, h->stream);
  sd.blk_beg = dupload(pl.s.blk_beg, *h->cur_owned, h->stream);
  sd.blk_end = dupload(pl.s.blk_end, *h->cur_owned, h->stream);
  sd.lvl_ptr = dupload(pl.s.lvl_ptr, *h->cur_owned, h->stream);
  d.d = sd;
  d.global_depth = pl.s.global_depth;
}

// fa() and fb() on two host threads; an exception of either is rethrown after both end.
template <typename FA, typename FB>
static void both(FA fa, FB fb) {
  std::exception_ptr ea, eb;
  std::thread t([&] {
    try {
      fa();
    } catch (...) {
      ea = std::current_exception();
    }
  });
  try {
    fb();
  } catch (...) {
    eb = std::current_exception();
  }
  t.join();
  if (ea) std::rethrow_exception(ea);
  if (eb) std::rethrow_exception(eb);
}

static void spmv_or_throw(cpc_solver* h, const MatDev& A, int mode, const void* x, bool xf32, const void* f,
                          bool ff32, void* y, bool yf32, int tpr, const int* done) {
  if (!launch_spmv(h->stream, A, mode, x, xf32, f, ff32, y, yf32, tpr, done))
    throw HipError{hipErrorInvalidValue, "unsupported SpMV precision combination"};
}

// fn(i) for i in [0, count) on up to `threads` host threads (fn must not throw).
template <typename F>
static void parallel_for(int count, int threads, F fn) {
  threads = std::max(1, std::min(threads, count));
  if (threads == 1) {
    for (int i = 0; i < count; ++i) fn(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&] {
      for (int i = next++; i < count; i = next++) fn(i);
    });
  for (auto& th : pool) th.join();
}

// Host threads for per-system setup work: the machine's, at most 16.
static int setup_threads() {
  const unsigned hc = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(hc ? hc : 1u, 16u));
}

// Upload the one-wave form of a triangular solve (wave_sweep.hip) over a wave
// schedule; share: a form over the same schedule and pattern whose step, row, slot and
// column arrays are reused (values differ). Not built (ok = 0) when no supported shape
// holds the longest row (more than 64 dependency entries).
// part_sys (batches): the batch system of each part of the schedule, for the per-system
// mask of the blocks.
static WaveDev upload_wave(cpc_solver* h, const HostCsr& a, const std::vector<double>& vals, const WaveSchedule& s,
                           const WaveDev* share, const std::vector<int>* part_sys = nullptr) {
  WaveDev w{};
  std::vector<std::pair<int, int>> shapes;
  // up to 64 dependency entries per row: longer rows (wide Galerkin levels) run faster
  // in the four-wave kernel, which keeps four times as many rows in flight per block
  for (int tb : {1, 2, 4, 8, 16})
    for (int k : {2, 4})
      if (wave_shape_supported(tb, k)) shapes.push_back({tb, k});
  WavePack wp;
  if (!build_wave_pack(a, vals, s, shapes, wp, setup_threads())) return w;
  if (wave_lds_bytes(wp.R, h->f32) > 150 * 1024) return w;
  if (share && share->ok && (share->tb != wp.tb || share->k != wp.k)) share = nullptr;
  w.ok = 1;
  w.tb = wp.tb;
  w.k = wp.k;
  w.nblk = wp.nblk;
  w.R = wp.R;
  w.W = s.W;
  w.M = s.M;
  w.nsteps = (int)wp.nsteps;
  w.grid = std::min(wp.nblk, 1024);
  if (share && share->ok) {
    w.blk_step = share->blk_step;
    w.col = share->col;
    w.row = share->row;
    w.slot = share->slot;
    w.mask = share->mask;
  } else {
    if (part_sys && (int)s.blk_part.size() == s.nblk) {
      std::vector<int> bs(s.nblk);
      bool okp = true;
      for (int t = 0; t < s.nblk; ++t) {
        const int p = s.blk_part[t];
        okp = okp && p >= 0 && p < (int)part_sys->size();
        bs[t] = okp ? (*part_sys)[p] : -1;
      }
      if (okp) w.mask.of = dupload(bs, *h->cur_owned, h->stream);
    }
    w.blk_step = dupload(wp.blk_step, *h->cur_owned, h->stream);
    w.col = dupload(wp.col, *h->cur_owned, h->stream);
    w.row = dupload(wp.row, *h->cur_owned, h->stream);
    w.slot = dupload(wp.slot, *h->cur_owned, h->stream);
  }
  if (h->f32) {
    w.val = dupload(std::vector<float>(wp.val.begin(), wp.val.end()), *h->cur_owned, h->stream);
    w.dinv = dupload(std::vector<float>(wp.dinv.begin(), wp.dinv.end()), *h->cur_owned, h->stream);
  } else {
    w.val = dupload(wp.val, *h->cur_owned, h->stream);
    w.dinv = dupload(wp.dinv, *h->cur_owned, h->stream);
  }
  return w;
}

// Segments per block of the one-wave form when the tuner has not chosen: four when the
// matrix's dominant coupling spans more than a block of R contiguous rows (the couplings
// between consecutive planes of a grid then stay inside a block), else one.
static int wave_segments(int stride, int R) { return stride >= R ? 4 : 1; }

// One-wave forms of the forward and backward solves of `a` (and of the ILU factor's,
// `lu` non-null) with R rows per block in M segments, into the packs given.
// Largest over the parts of each part's dominant coupling distance.
static int parts_stride(const HostCsr& a, const std::vector<int>& parts) {
  const int np = (int)parts.size() - 1;
  std::vector<int> mode(std::max(np, 0), 0);
  parallel_for(np, setup_threads(), [&](int p) {
    std::map<int, int> count;
    for (int i = parts[p]; i < parts[p + 1]; ++i)
      if (a.rp[i] < a.rp[i + 1] && a.ci[a.rp[i]] < i) ++count[i - a.ci[a.rp[i]]];
    int mc = 0;
    for (const auto& kv : count)
      if (kv.second > mc) {
        mode[p] = kv.first;
        mc = kv.second;
      }
  });
  int best = 0;
  for (int m : mode) best = std::max(best, m);
  return best;
}

// One-wave forms of the forward and backward solves of `a` (and of the ILU factor's,
// `lu` non-null) with R rows per block in M segments, each system of `parts` scheduled
// on its own (the two directions built on two host threads), into the packs given.
// Returns true when every form was built; depth_lo / depth_up receive the schedules'
// numbers of level sets.
static bool build_wave_forms(cpc_solver* h, const HostCsr& a, int R, int M, const std::vector<int>& parts,
                             SweepPackDev& lo, SweepPackDev& up, const std::vector<double>* lu, SweepPackDev* ilo,
                             SweepPackDev* iup, int* depth_lo, int* depth_up,
                             const std::vector<int>* part_sys = nullptr) {
  if (h->opt.sweep_kernel == 1) return false;
  const int W = std::max(1, R / std::max(1, M));
  const int threads = std::max(1, setup_threads() / 2);
  WaveSchedule wl, wu;
  std::thread tl([&] { build_wave_schedule_parts(a, true, W, M, parts, threads, wl); });
  build_wave_schedule_parts(a, false, W, M, parts, threads, wu);
  tl.join();
  lo.wave = upload_wave(h, a, a.v, wl, nullptr, part_sys);
  up.wave = upload_wave(h, a, a.v, wu, nullptr, part_sys);
  bool all = lo.wave.ok && up.wave.ok;
  if (lu && ilo && iup) {
    ilo->wave = upload_wave(h, a, *lu, wl, &lo.wave);
    iup->wave = upload_wave(h, a, *lu, wu, &up.wave);
    all = all && ilo->wave.ok && iup->wave.ok;
  }
  if (depth_lo) *depth_lo = wl.global_depth;
  if (depth_up) *depth_up = wu.global_depth;
  return all;
}

// The rows of a triangular solve packed in its processing order (host side): the
// dependency entries (left of the diagonal forward, right of it backward) with columns
// in the row's own block stored block-relative and the others as -(j + 1).
struct PackHost {
  std::vector<int> ptr, col;
  std::vector<double> diag, v;
  int tb = 1;
};
static PackHost pack_host(const HostCsr& a, const std::vector<double>& vals, const SweepSchedule& s) {
  PackHost ph;
  const int n = a.n;
  const bool fwd = s.forward;
  const int nt = setup_threads();
  std::vector<int>& ptr = ph.ptr;
  std::vector<double>& diag = ph.diag;  // reciprocal diagonal
  ptr.assign(n + 1, 0);
  diag.assign(n, 1.0);
  chunked(n, nt, 65536, [&](int64_t p0, int64_t p1) {
    for (int64_t p = p0; p < p1; ++p) {
      const int i = s.perm[p];
      int c = 0;
      for (int q = a.rp[i]; q < a.rp[i + 1]; ++q) {
        const int j = a.ci[q];
        if (j == i) diag[p] = 1.0 / vals[q];
        else if (fwd ? j < i : j > i) ++c;
      }
      ptr[p + 1] = c;
    }
  });
  for (int p = 0; p < n; ++p) ptr[p + 1] += ptr[p];
  const int64_t ne = ptr[n];
  std::vector<int>& col = ph.col;
  std::vector<double>& v = ph.v;
  col.assign((size_t)std::max<int64_t>(ne, 1), 0);
  v.assign((size_t)std::max<int64_t>(ne, 1), 0.0);
  {
    std::vector<int> blk_of(n);
    chunked(s.nblk, nt, 16, [&](int64_t b0, int64_t b1) {
      for (int64_t b = b0; b < b1; ++b)
        for (int i = s.blk_row[b]; i < s.blk_row[b + 1]; ++i) blk_of[i] = (int)b;
    });
    chunked(n, nt, 65536, [&](int64_t p0, int64_t p1) {
      for (int64_t p = p0; p < p1; ++p) {
        const int i = s.perm[p];
        const int b = blk_of[i];
        int w = ptr[p];
        for (int q = a.rp[i]; q < a.rp[i + 1]; ++q) {
          const int j = a.ci[q];
          if (j == i || !(fwd ? j < i : j > i)) continue;
          col[w] = (blk_of[j] == b) ? j - s.blk_row[b] : -(j + 1);
          v[w] = vals[q];
          ++w;
        }
      }
    });
  }
  // lanes per row in the summing phase: about eight products per lane
  const double avg = n ? (double)ne / n : 0.0;
  int t = 1;
  while (t < 64 && t * 8 < avg) t <<= 1;
  ph.tb = t;
  return ph;
}

// share: reuse the row/ptr/col arrays of a pack with the same schedule and direction
// (values differ).
static SweepPackDev upload_pack(cpc_solver* h, const PackHost& ph, const SweepSchedule& s,
                                const SweepPackDev* share) {
  SweepPackDev pk{};
  if (share) {
    pk.row = share->row;
    pk.ptr = share->ptr;
    pk.col = share->col;
  } else {
    pk.row = dupload(s.perm, *h->cur_owned, h->stream);
    pk.ptr = dupload(ph.ptr, *h->cur_owned, h->stream);
    pk.col = dupload(ph.col, *h->cur_owned, h->stream);
  }
  if (h->f32) {
    std::vector<float> v32(ph.v.begin(), ph.v.end()), d32(ph.diag.begin(), ph.diag.end());
    pk.val = dupload(v32, *h->cur_owned, h->stream);
    pk.diag = dupload(d32, *h->cur_owned, h->stream);
  } else {
    pk.val = dupload(ph.v, *h->cur_owned, h->stream);
    pk.diag = dupload(ph.diag, *h->cur_owned, h->stream);
  }
  pk.tb = ph.tb;
  return pk;
}

// Schedules and packs of both directions of the four-wave kernel (the host work of the
// two directions on two threads), and those of a second factor on the same schedules
// (lu non-null: the ILU(0) values).
static void build_fourwave(cpc_solver* h, const HostCsr& a, int R, DevSweepSched& lo, DevSweepSched& up,
                           SweepPackDev& fl, SweepPackDev& fu, const std::vector<double>* lu, SweepPackDev* il,
                           SweepPackDev* iu, const std::vector<int>* parts = nullptr,
                           const std::vector<int>* part_sys = nullptr) {
  SweepPlan pl, pu;
  PackHost hl, hu, hil, hiu;
  both([&] {
         pl = plan_sweep(h, a, true, R, parts);
         hl = pack_host(a, a.v, pl.s);
         if (lu) hil = pack_host(a, *lu, pl.s);
       },
       [&] {
         pu = plan_sweep(h, a, false, R, parts);
         hu = pack_host(a, a.v, pu.s);
         if (lu) hiu = pack_host(a, *lu, pu.s);
       });
  upload_sweep(h, pl, lo, parts, part_sys);
  upload_sweep(h, pu, up, parts, part_sys);
  fl = upload_pack(h, hl, pl.s, nullptr);
  fu = upload_pack(h, hu, pu.s, nullptr);
  if (lu && il && iu) {
    *il = upload_pack(h, hil, pl.s, &fl);
    *iu = upload_pack(h, hiu, pu.s, &fu);
  }
}

// The per-system mask of a batched solve over a launch's unit map (no mask outside a
// batched solve or without a map).
static SysMask mask_of(const cpc_solver* h, const int* of) {
  SysMask m;
  if (h->mask_done && of) {
    m.of = of;
    m.done = h->mask_done;
  }
  return m;
}
static MatDev masked_rows(const cpc_solver* h, MatDev m, const int* row_sys) {
  m.mask = mask_of(h, row_sys);
  return m;
}
static DenseTriDev dmask(const cpc_solver* h, DenseTriDev dt) {
  dt.mask = mask_of(h, dt.mask.of);
  return dt;
}
static DenseListDev lmask(const cpc_solver* h, DenseListDev dl) {
  dl.mask = mask_of(h, dl.mask.of);
  return dl;
}

// x = T^{-1} f for the triangular factor the pack holds (out = base + x for
// SWEEP_UPPER_OUT). x is first filled with the not-yet-solved marker.
// The triangular-solve kernel of a pack: the one-wave form where the pack has it, else
// the four-wave workgroup kernel. x must hold the sentinel.
// ev0 / ev1 (measurement only): events that end up holding the kernel's start and end.
static void launch_tri(cpc_solver* h, int op, const DevSweepSched& sch, const SweepPackDev& pk, const void* f,
                       void* x, const void* base, void* out, const int* done, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr) {
  if (pk.wave.ok) {
    WaveDev w = pk.wave;
    w.mask = mask_of(h, w.mask.of);
    launch_wave_sweep(h->stream, op, w, h->f32, f, x, base, out, h->sync, done, h->spin_limit, ev0, ev1);
  } else {
    SweepDev sd = sch.d;
    sd.mask = mask_of(h, sd.mask.of);
    if (ev0) HIPCHK(hipEventRecord(ev0, h->stream));
    launch_sweep_packed(h->stream, op, sd, pk, h->f32, f, x, base, out, h->sync, done, h->spin_limit);
    if (ev1) HIPCHK(hipEventRecord(ev1, h->stream));
  }
}

static void run_sweep(cpc_solver* h, int op, const DevSweepSched& sch, const SweepPackDev& pk, const void* f,
                      void* x, const void* base, void* out, const int* done) {
  launch_fill_sentinel(h->stream, sch.d.n, x, h->f32, done);
  launch_tri(h, op, sch, pk, f, x, base, out, done);
}

// Strict lower triangle of a (the old-value part of a backward Gauss-Seidel sweep).
static HostCsr strict_lower(const HostCsr& a) {
  HostCsr t;
  t.n = a.n;
  t.ncols = a.ncols;
  t.rp.assign(a.n + 1, 0);
  const int nt = setup_threads();
  chunked(a.n, nt, 65536, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      int c = 0;
      for (int q = a.rp[i]; q < a.rp[i + 1]; ++q) c += a.ci[q] < i;
      t.rp[i + 1] = c;
    }
  });
  for (int i = 0; i < a.n; ++i) t.rp[i + 1] += t.rp[i];
  t.ci.resize(t.rp[a.n]);
  t.v.resize(t.rp[a.n]);
  chunked(a.n, nt, 65536, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      int w = t.rp[i];
      for (int q = a.rp[i]; q < a.rp[i + 1]; ++q)
        if (a.ci[q] < i) {
          t.ci[w] = a.ci[q];
          t.v[w++] = a.v[q];
        }
    }
  });
  return t;
}

// A matrix of nrows x ncols made of blocks placed at row and column offsets; the
// blocks' row ranges tile [0, nrows). Blocks are copied on host threads.
struct PlacedBlock {
  const HostCsr* m;
  int row_off, col_off;
};
static void place_blocks(std::vector<PlacedBlock> blocks, int nrows, int ncols, HostCsr& out) {
  std::sort(blocks.begin(), blocks.end(),
            [](const PlacedBlock& x, const PlacedBlock& y) { return x.row_off < y.row_off; });
  std::vector<int64_t> nz(blocks.size() + 1, 0);
  for (size_t k = 0; k < blocks.size(); ++k) nz[k + 1] = nz[k] + blocks[k].m->nnz();
  out.n = nrows;
  out.ncols = ncols;
  out.rp.assign(nrows + 1, 0);
  out.ci.resize(nz.back());
  out.v.resize(nz.back());
  parallel_for((int)blocks.size(), setup_threads(), [&](int k) {
    const HostCsr& m = *blocks[k].m;
    const int r0 = blocks[k].row_off, c0 = blocks[k].col_off;
    const int64_t base = nz[k];
    for (int i = 0; i < m.n; ++i) out.rp[r0 + i + 1] = (int)(base + m.rp[i + 1]);
    for (int64_t q = 0; q < (int64_t)m.ci.size(); ++q) {
      out.ci[base + q] = m.ci[q] + c0;
      out.v[base + q] = m.v[q];
    }
  });
}

// ---------------------------------------------------------------------------
// Preconditioner application (all asynchronous on h->stream).

// One system's hierarchy, built on its own (host splitting and interpolation, GPU
// Galerkin products in temporary device buffers).
struct SysHier {
  std::vector<HostCsr> A;             // A_l for depth 0 .. L-1
  std::vector<HostCsr> P;             // P for depth d -> d+1
  std::vector<std::vector<int>> cf;   // C/F splitting of each split depth
  std::vector<double> lu;             // ILU(0) values on A[0]
  std::vector<double> inv;            // dense inverse of A[L-1]
};

// stream: where its Galerkin products run (null: the handle's stream); the host parts
// touch only S, so systems of a batch can be built on threads of their own.
static int build_sys_hier(cpc_solver* h, SysHier& S, const cpc_options& o, std::string* msg,
                          hipStream_t stream = nullptr) {
  const hipStream_t hs = stream ? stream : h->stream;
  std::vector<void*> tmp;
  int status = CPC_OK;
  try {
    DevCsr Ad;
    upload_csr(h, S.A[0], Ad, false, &tmp, false, hs);
    for (int d = 0;; ++d) {
      const HostCsr& A = S.A[d];
      if (A.n <= o.max_coarse || d + 1 >= o.max_levels) break;
      std::vector<int> cf;
      const int nc = rs_coarsen(A, o.theta, cf);
      if (nc == 0 || (double)nc > 0.9 * (double)A.n) break;
      HostCsr P;
      rs_interpolation(A, o.theta, cf, nc, P);
      HostCsr R = transpose(P);
      DevCsr Pd, Rd, APd, Acd;
      upload_csr(h, P, Pd, false, &tmp, false, hs);
      upload_csr(h, R, Rd, false, &tmp, false, hs);
      HostCsr AP, Ac;
      if (!gpu_spgemm(h, Ad, Pd, nc, AP, APd, msg, tmp, hs) || !gpu_spgemm(h, Rd, APd, nc, Ac, Acd, msg, tmp, hs)) {
        status = CPC_E_NOMEM;
        break;
      }
      for (int i = 0; i < Ac.n; ++i) {
        bool diag = false;
        for (int k = Ac.rp[i]; k < Ac.rp[i + 1]; ++k) diag |= (Ac.ci[k] == i);
        if (!diag) {
          if (msg) *msg = "coarse matrix lost its diagonal";
          status = CPC_E_NOT_SPD;
          break;
        }
      }
      if (status != CPC_OK) break;
      S.cf.push_back(std::move(cf));
      S.P.push_back(std::move(P));
      S.A.push_back(std::move(Ac));
      Ad = Acd;
    }
    if (status == CPC_OK) {
      const HostCsr& Lc = S.A.back();
      if (Lc.n > 8192) {
        if (msg) *msg = "coarsening stalled with " + std::to_string(Lc.n) + " rows";
        status = CPC_E_NOMEM;
      } else {
        status = dense_spd_inverse(Lc, S.inv, msg);
      }
    }
    HIPCHK(hipStreamSynchronize(hs));
  } catch (...) {
    (void)hipStreamSynchronize(hs);
    for (void* p : tmp) (void)hipFree(p);
    throw;
  }
  for (void* p : tmp) (void)hipFree(p);
  return status;
}

// Explicit inverses of T = D + L for the smoothed systems of a level (all of them or
// none): at most 16384 rows each (larger levels take the block form) and 64 GB. The
// row products address one system's inverse with 32-bit byte offsets, which holds up to
// 16384 rows (2 GiB in FP64); diagonal blocks of the block form obey the same limit.
static constexpr int kDenseMaxRows = 16384;
// Device memory one level's block form (inverses and their transposes) may take: at
// most 96 GB and 60 % of what is free when it is built (a level of 1.4 M rows in
// 4096-row blocks on an MI355X's 288 GB; later levels see what earlier ones left).
static double blockdense_cap() {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    return 32e9;
  }
  return std::min(96e9, 0.6 * (double)free_b);
}

// Sum of the squares of the block sizes of the block form with B-row blocks over the
// row ranges `parts` (each cut on its own, the last block of a range short). The form
// stores each block's inverse and its transpose as FP64 squares first (16 bytes per
// entry of the sum: the memory bound), and one forward plus one backward solve reads
// the lower triangle of the one and the upper triangle of the other, at least an
// entry's width per entry of the sum, so at the HBM peak of 8 TB/s that pair takes at
// least width x sum / 8e12 seconds.
static double blockdense_squares(const std::vector<int>& parts, int B) {
  double sq = 0.0;
  for (size_t p = 0; p + 1 < parts.size(); ++p) {
    const double s = parts[p + 1] - parts[p];
    const double full = std::floor(s / B), tail = s - full * B;
    sq += full * B * (double)B + tail * tail;
  }
  return sq;
}
static constexpr double kDenseMaxBytes = 64e9;
static constexpr int kDenseTransRows = 16384;

// Scratch of dense_tri_inverse for n rows: the products W = B A^{-1} of all pairs of
// one span length at once (sp x sp each, the last pair's rows fewer).
static long dense_work_need(int n) {
  long w = 1;
  for (int sp = 128; sp < n; sp *= 2) {
    long t = 0;
    for (int a = 0; a + sp < n; a += 2 * sp) t += (long)sp * (std::min(a + 2 * sp, n) - a - sp);
    w = std::max(w, t);
  }
  return w;
}

static void build_dense(cpc_solver* h, Level& L, const std::vector<int>& ns, const std::vector<int>& voffs) {
  if (h->opt.dense_smoother == 1 || h->opt.dense_smoother == 3 || ns.empty()) return;
  double bytes = 0.0;
  for (int n : ns) {
    if (n > kDenseMaxRows) return;
    bytes += 8.0 * n * (double)n;
  }
  if (bytes > kDenseMaxBytes) return;
  std::vector<long> moff(ns.size());
  long tot = 0, wmax = 1;
  for (size_t k = 0; k < ns.size(); ++k) {
    moff[k] = tot;
    tot += (long)ns[k] * dense_ld(ns[k]);
    wmax = std::max(wmax, dense_work_need(ns[k]));
  }
  double* M64 = nullptr;
  double* work = nullptr;
  if (hipMalloc(&M64, sizeof(double) * tot) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  if (hipMalloc(&work, sizeof(double) * wmax) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(M64);
    return;
  }
  bool ok = true;
  std::string msg;
  for (size_t k = 0; ok && k < ns.size(); ++k)
    ok = dense_tri_inverse(h->stream, ns[k], voffs[k], L.A.rp, L.A.ci, L.A.v, M64 + moff[k], work, &msg);
  ok = ok && hipStreamSynchronize(h->stream) == hipSuccess;
  (void)hipFree(work);
  if (!ok) {
    (void)hipGetLastError();
    (void)hipFree(M64);
    return;
  }
  void* M = M64;
  if (h->f32) {
    float* M32 = nullptr;
    if (hipMalloc(&M32, sizeof(float) * tot) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(M64);
      return;
    }
    launch_to_type(h->stream, tot, M64, M32, true);
    HIPCHK(hipStreamSynchronize(h->stream));
    (void)hipFree(M64);
    M = M32;
  }
  std::vector<int4> itn, itt, red;
  int slot = 0;
  double ent = 0.0;
  for (int k = 0; k < (int)ns.size(); ++k) {
    const int n = ns[k];
    ent += 0.5 * (double)n * (n + 1);
    dense_row_items(k, n, itn);
    for (int c0 = 0; c0 < n; c0 += kTCols) {
      const int first = slot;
      for (int r0 = (c0 / kTChunk) * kTChunk; r0 < n; r0 += kTChunk) itt.push_back(make_int4(k, c0, r0, slot++));
      red.push_back(make_int4(k, c0, first, slot - first));
    }
  }
  DenseTriDev& dt = L.dtri;
  dt.max_n = *std::max_element(ns.begin(), ns.end());
  dt.n = dupload(ns, h->owned, h->stream);
  dt.moff = dupload(moff, h->owned, h->stream);
  dt.voff = dupload(voffs, h->owned, h->stream);
  dt.M = M;
  dt.nitem_n = (int)itn.size();
  dt.item_n = dupload(itn, h->owned, h->stream);
  if (ns.size() == 1) {
    dt.one_n = ns[0];
    dt.one_voff = voffs[0];
    dt.one_moff = moff[0];
    dt.one_sys = 0;
  }
  if (h->batch && L.part_sys.size() == ns.size()) dt.mask.of = dupload(L.part_sys, h->owned, h->stream);
  dt.nitem_t = (int)itt.size();
  dt.item_t = dupload(itt, h->owned, h->stream);
  dt.nred = (int)red.size();
  dt.red = dupload(red, h->owned, h->stream);
  dt.part = dalloc<double>((size_t)slot * kTCols, h->owned);
  // systems of at most 16384 rows also keep the transpose (row products both ways)
  bool small = true;
  for (int n : ns) small = small && n <= kDenseTransRows;
  if (small) {
    const size_t es = h->f32 ? sizeof(float) : sizeof(double);
    void* MTr = nullptr;
    if (hipMalloc(&MTr, es * tot) == hipSuccess) {
      HIPCHK(hipMemsetAsync(MTr, 0, es * tot, h->stream));  // zero padding columns
      for (size_t k = 0; k < ns.size(); ++k)
        launch_transpose(h->stream, ns[k], (const char*)M + es * moff[k], (char*)MTr + es * moff[k], h->f32);
      HIPCHK(hipStreamSynchronize(h->stream));
      dt.MT = MTr;
      L.dense_MT = MTr;
    } else {
      (void)hipGetLastError();
    }
  }
  L.dense_M = M;
  L.dense_entries = ent;
  L.dense_bytes = (double)(h->f32 ? sizeof(float) : sizeof(double)) * (double)tot * (dt.MT ? 2.0 : 1.0);
}

// Iterations to launch before the next read of the convergence state when no fixed
// count is set: the mean residual reduction per iteration so far predicts how many
// remain, and three quarters of that (at least one, at most 64) are launched, so a solve
// rarely replays an iteration past convergence (a full graph of launches that return at
// once) and reads the state a few times instead of after every iteration.
static int predicted_chunk(const PcgState& hs, int it0, double rel0) {
  const int done_its = hs.iters - it0;
  if (done_its < 1 || !(rel0 > 0.0) || !(hs.relres > 0.0) || !(hs.tol > 0.0) || !(hs.relres > hs.tol)) return 1;
  const double q = std::pow(hs.relres / rel0, 1.0 / done_its);
  if (!(q > 0.0 && q < 1.0)) return 1;
  const double m = std::log(hs.tol / hs.relres) / std::log(q);
  if (!(m > 0.0)) return 1;
  return std::max(1, std::min(64, (int)(0.75 * m)));
}

// Average milliseconds of fn() over reps launches after one warm-up (events on the
// handle's stream).
template <typename F>
static float time_ms(cpc_solver* h, int reps, F fn) {
  fn();
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, h->stream));
  for (int r = 0; r < reps; ++r) fn();
  HIPCHK(hipEventRecord(e1, h->stream));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

// Keep each level's explicit inverse only where it smooths faster than the sweeps
// (measured on the handle's own matrices), or everywhere it was built when asked to.
static void tune_dense(cpc_solver* h) {
  const bool f32 = h->f32;
  for (size_t d = 0; d < h->lev.size(); ++d) {
    Level& L = h->lev[d];
    if (!L.dense_M) continue;
    bool keep = h->opt.dense_smoother == 2 || (!h->opt.tune && L.A.n <= 8192);
    if (!keep && h->opt.tune) {
      void* f = d == 0 ? h->pin : L.f;
      void* u = d == 0 ? h->u1 : L.u;
      const float ts = time_ms(h, 3, [&] {
        run_sweep(h, SWEEP_LOWER, L.lower, L.fgs, f, u, nullptr, nullptr, nullptr);
        run_sweep(h, SWEEP_UPPER, L.upper, L.bgs, f, u, nullptr, nullptr, nullptr);
      });
      const float td = time_ms(h, 3, [&] {
        launch_dense_lower(h->stream, L.dtri, f32, f32, f, u, nullptr);
        launch_dense_lower_t(h->stream, L.dtri, f32, f32, f, u, nullptr);
      });
      keep = td < ts;
    }
    if (keep) {
      L.dense_owned.push_back(L.dense_M);
      if (L.dense_MT) L.dense_owned.push_back(L.dense_MT);
      L.dense_smooth = true;
    } else {
      (void)hipFree(L.dense_M);
      if (L.dense_MT) (void)hipFree(L.dense_MT);
      L.dtri = DenseTriDev{};
      L.dense_entries = 0.0;
    }
    L.dense_M = nullptr;
    L.dense_MT = nullptr;
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  unsigned herr = 0;
  HIPCHK(hipMemcpy(&herr, h->sync.err, sizeof(unsigned), hipMemcpyDeviceToHost));
  if (herr) throw HipError{hipErrorUnknown, "a sweep wait exceeded its bound while tuning"};
}

// Schedules and packed rows of a level's triangular solves with blocks of R rows
// (and the ILU(0) packs on the finest level), allocated in the level's own list.
static void build_level_sweeps(cpc_solver* h, Level& L, const HostCsr& sub, int R, bool ilu) {
  std::vector<void*>* prev = h->cur_owned;
  h->cur_owned = &L.sweep_owned;
  try {
    const bool with_ilu = ilu && !h->iluk;
    const std::vector<int> parts =
        (!L.parts.empty() && L.parts.front() == 0 && L.parts.back() == sub.n) ? L.parts : std::vector<int>{0, sub.n};
    if (L.wave_stride < 0) L.wave_stride = parts_stride(sub, parts);
    const int M = L.wave_M > 0 ? L.wave_M : wave_segments(L.wave_stride, R);
    SweepPackDev fw{}, bw{}, ilw{}, iuw{};
    int dlo = 0, dup = 0;
    const std::vector<int>* psys =
        (h->batch && L.part_sys.size() + 1 == parts.size() && parts.size() > 1) ? &L.part_sys : nullptr;
    const bool wave_all =
        build_wave_forms(h, sub, R, M, parts, fw, bw, with_ilu ? &h->lu_host : nullptr,
                                        with_ilu ? &ilw : nullptr, with_ilu ? &iuw : nullptr, &dlo, &dup, psys);
    if (wave_all) {
      // the one-wave forms serve every solve of the level: no four-wave schedules
      L.lower = DevSweepSched{};
      L.upper = DevSweepSched{};
      L.lower.d.n = L.upper.d.n = sub.n;
      L.lower.global_depth = dlo;
      L.upper.global_depth = dup;
      L.fgs = fw;
      L.bgs = bw;
      if (with_ilu) {
        h->ilu_l = ilw;
        h->ilu_u = iuw;
      }
    } else {
      const int Rw = std::min(R, sweep_max_rows_per_block());  // the four-wave kernel's blocks
      build_fourwave(h, sub, Rw, L.lower, L.upper, L.fgs, L.bgs, with_ilu ? &h->lu_host : nullptr,
                     with_ilu ? &h->ilu_l : nullptr, with_ilu ? &h->ilu_u : nullptr, h->batch ? &parts : nullptr,
                     psys);
      L.fgs.wave = fw.wave;
      L.bgs.wave = bw.wave;
      if (with_ilu) {
        h->ilu_l.wave = ilw.wave;
        h->ilu_u.wave = iuw.wave;
      }
    }
  } catch (...) {
    h->cur_owned = prev;
    throw;
  }
  h->cur_owned = prev;
  L.sweep_R = R;
}

// Schedules and packs of an ILU(k) factor with k > 0 (its pattern is not that of A, so
// the triangular solves of B get their own), rows per block R; built once after the
// level-0 sweeps are settled.
static void build_iluk_sweeps(cpc_solver* h, int R) {
  std::vector<void*>* prev = h->cur_owned;
  h->cur_owned = &h->owned;
  try {
    const std::vector<int> parts{0, h->iluF.n};
    const int stride = parts_stride(h->iluF, parts);
    SweepPackDev lw{}, uw{};
    int dlo = 0, dup = 0;
    if (build_wave_forms(h, h->iluF, R, wave_segments(stride, R), parts, lw, uw, nullptr, nullptr, nullptr, &dlo,
                         &dup)) {
      h->ilu_lower = DevSweepSched{};
      h->ilu_upper = DevSweepSched{};
      h->ilu_lower.d.n = h->ilu_upper.d.n = h->iluF.n;
      h->ilu_lower.global_depth = dlo;
      h->ilu_upper.global_depth = dup;
      h->ilu_l = lw;
      h->ilu_u = uw;
    } else {
      const int Rw = std::min(R, sweep_max_rows_per_block());
      build_fourwave(h, h->iluF, Rw, h->ilu_lower, h->ilu_upper, h->ilu_l, h->ilu_u, nullptr, nullptr, nullptr);
      h->ilu_l.wave = lw.wave;
      h->ilu_u.wave = uw.wave;
    }
  } catch (...) {
    h->cur_owned = prev;
    throw;
  }
  h->cur_owned = prev;
}

// The schedules the ILU triangular solves run on.
static const DevSweepSched& ilu_lower_sched(const cpc_solver* h) { return h->iluk ? h->ilu_lower : h->lev[0].lower; }
static const DevSweepSched& ilu_upper_sched(const cpc_solver* h) { return h->iluk ? h->ilu_upper : h->lev[0].upper; }

// Block-dense form of a level's Gauss-Seidel factor T = D + L with blocks of B rows
// (each system of a batch cut on its own): the forward solve is, block by block,
// g_b = f_b - (T entries left of the block) x, x_b = T_bb^{-1} g_b; the backward solve
// with T^T = D + U runs each system's blocks in reverse with the entries right of the
// block and x_b = T_bb^{-T} g_b. Blocks of different systems are independent, so each
// step takes one block of every system. Returns false (nothing kept) when the inverses
// do not fit or a step fails.
static bool build_blockdense(cpc_solver* h, Level& L, const HostCsr& sub, int B) {
  if (B <= 0 || B > kDenseMaxRows) return false;
  const int n = sub.n;
  const std::vector<int> parts =
      (!L.parts.empty() && L.parts.front() == 0 && L.parts.back() == n) ? L.parts : std::vector<int>{0, n};
  const int np = (int)parts.size() - 1;
  BlockDense bd;
  bd.B = B;
  std::vector<int> kc(np);
  int kmax = 0;
  for (int p = 0; p < np; ++p) {
    kc[p] = (parts[p + 1] - parts[p] + B - 1) / B;
    kmax = std::max(kmax, kc[p]);
  }
  std::vector<std::vector<int>> id(np);  // block index of the k-th block of part p
  const bool with_sys = h->batch && (int)L.part_sys.size() == np;
  std::vector<int> blk_sys;  // batch system of each block (per-system mask)
  bd.fstep.push_back(0);
  for (int k = 0; k < kmax; ++k) {
    for (int p = 0; p < np; ++p) {
      if (k >= kc[p]) continue;
      id[p].push_back(bd.nblk());
      if (with_sys) blk_sys.push_back(L.part_sys[p]);
      const int r0 = parts[p] + k * B;
      bd.start.push_back(r0);
      bd.rows.push_back(std::min(B, parts[p + 1] - r0));
    }
    bd.fstep.push_back(bd.nblk());
  }
  bd.bstep.push_back(0);
  for (int t = 0; t < kmax; ++t) {
    for (int p = 0; p < np; ++p)
      if (t < kc[p]) bd.bblk.push_back(id[p][kc[p] - 1 - t]);
    bd.bstep.push_back((int)bd.bblk.size());
  }
  const int K = bd.nblk();
  double bytes = 0.0;
  for (int b = 0; b < K; ++b) bytes += 16.0 * bd.rows[b] * (double)bd.rows[b];
  if (bytes > blockdense_cap()) return false;
  // entries outside each row's block, rows in step order (forward: left of the block;
  // backward: right of it)
  HostCsr lo, up;
  std::vector<int> lrid, urid;
  lo.ncols = up.ncols = sub.ncols;
  lo.rp.assign(1, 0);
  up.rp.assign(1, 0);
  auto add_rows = [&](HostCsr& m, std::vector<int>& rid, int b, bool left) {
    const int b0 = bd.start[b], b1 = b0 + bd.rows[b];
    for (int i = b0; i < b1; ++i) {
      for (int q = sub.rp[i]; q < sub.rp[i + 1]; ++q) {
        const int j = sub.ci[q];
        if (left ? j < b0 : j >= b1) {
          m.ci.push_back(j);
          m.v.push_back(sub.v[q]);
        }
      }
      m.rp.push_back((int)m.ci.size());
      rid.push_back(i);
    }
  };
  bd.frow.push_back(0);
  for (int k = 0; k < kmax; ++k) {
    for (int b = bd.fstep[k]; b < bd.fstep[k + 1]; ++b) add_rows(lo, lrid, b, true);
    bd.frow.push_back((int)lrid.size());
  }
  bd.brow.push_back(0);
  for (int t = 0; t < kmax; ++t) {
    for (int q = bd.bstep[t]; q < bd.bstep[t + 1]; ++q) add_rows(up, urid, bd.bblk[q], false);
    bd.brow.push_back((int)urid.size());
  }
  lo.n = (int)lrid.size();
  up.n = (int)urid.size();
  std::vector<void*>& own = bd.owned;
  long tot = 0, wmax = 1;
  bd.moff.resize(K);
  for (int b = 0; b < K; ++b) {
    bd.moff[b] = tot;
    tot += (long)bd.rows[b] * dense_ld(bd.rows[b]);
    wmax = std::max(wmax, dense_work_need(bd.rows[b]));
  }
  auto drop = [&] {
    (void)hipStreamSynchronize(h->stream);
    for (void* p : own) (void)hipFree(p);
    (void)hipGetLastError();
    return false;
  };
  double* M64 = nullptr;
  double* work = nullptr;
  if (hipMalloc(&M64, sizeof(double) * tot) != hipSuccess) return drop();
  if (hipMalloc(&work, sizeof(double) * wmax) != hipSuccess) {
    (void)hipFree(M64);
    return drop();
  }
  bool ok = true;
  std::string msg;
  for (int b = 0; ok && b < K; ++b)
    ok = dense_tri_inverse(h->stream, bd.rows[b], bd.start[b], L.A.rp, L.A.ci, L.A.v, M64 + bd.moff[b], work, &msg);
  ok = ok && hipStreamSynchronize(h->stream) == hipSuccess;
  (void)hipFree(work);
  if (!ok) {
    (void)hipFree(M64);
    return drop();
  }
  const size_t es = h->f32 ? sizeof(float) : sizeof(double);
  void* M = M64;
  if (h->f32) {
    float* M32 = nullptr;
    if (hipMalloc(&M32, sizeof(float) * tot) != hipSuccess) {
      (void)hipFree(M64);
      return drop();
    }
    launch_to_type(h->stream, tot, M64, M32, true);
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(M64);
    M = M32;
  }
  own.push_back(M);
  void* MT = nullptr;
  if (hipMalloc(&MT, es * tot) != hipSuccess) return drop();
  own.push_back(MT);
  if (hipMemsetAsync(MT, 0, es * tot, h->stream) != hipSuccess) return drop();  // zero padding columns
  for (int b = 0; b < K; ++b)
    launch_transpose(h->stream, bd.rows[b], (const char*)M + es * bd.moff[b], (char*)MT + es * bd.moff[b], h->f32);
  bd.stored_bytes = 2.0 * (double)es * (double)tot;
  // row items of each step, the forward steps' and the backward steps' in lists of their own
  std::vector<int4> itf, itb;
  bd.fitem.push_back(0);
  for (int k = 0; k < kmax; ++k) {
    for (int b = bd.fstep[k]; b < bd.fstep[k + 1]; ++b) dense_row_items(b, bd.rows[b], itf);
    bd.fitem.push_back((int)itf.size());
  }
  bd.bitem.push_back(0);
  for (int t = 0; t < kmax; ++t) {
    for (int q = bd.bstep[t]; q < bd.bstep[t + 1]; ++q) dense_row_items(bd.bblk[q], bd.rows[bd.bblk[q]], itb);
    bd.bitem.push_back((int)itb.size());
  }
  for (int b = 0; b < K; ++b) bd.entries += 0.5 * (double)bd.rows[b] * (bd.rows[b] + 1);
  try {
    upload_csr(h, lo, bd.Loff, false, &own);
    upload_csr(h, up, bd.Uoff, false, &own);
    bd.Lrid = dupload(lrid, own, h->stream);
    bd.Urid = dupload(urid, own, h->stream);
    // a step's off-block product over one block is a small launch that ends with its
    // longest row: lanes enough for that row to take a single batch of four entries per
    // lane. Steps over many blocks (batches) have rows enough to keep the GPU busy: lanes
    // by the average row, as for any large SpMV.
    for (auto* m : {&lo, &up}) {
      int longest = 0;
      for (int i = 0; i < m->n; ++i) longest = std::max(longest, m->rp[i + 1] - m->rp[i]);
      DevCsr& d = m == &lo ? bd.Loff : bd.Uoff;
      const double rows_per_step = kmax > 0 ? (double)m->n / kmax : 0.0;
      if (rows_per_step > 16384.0) {
        const double avg = m->n ? (double)m->rp[m->n] / m->n : 1.0;
        d.tpr = pick_tpr(avg);
        d.steps = pick_steps(avg, d.tpr);
      } else {
        d.tpr = 1;
        while (d.tpr < 64 && 4 * d.tpr < longest) d.tpr <<= 1;
        d.steps = 4;
      }
    }
    DenseTriDev& dt = bd.dt;
    dt = DenseTriDev{};
    dt.n = dupload(bd.rows, own, h->stream);
    dt.moff = dupload(bd.moff, own, h->stream);
    dt.voff = dupload(bd.start, own, h->stream);
    dt.M = M;
    dt.MT = MT;
    bd.items_f = dupload(itf, own, h->stream);
    bd.items_b = dupload(itb, own, h->stream);
    if (with_sys) dt.mask.of = dupload(blk_sys, own, h->stream);
    HIPCHK(hipStreamSynchronize(h->stream));
  } catch (const HipError&) {
    return drop();
  }
  L.bd = std::move(bd);
  return true;
}

static void free_blockdense(cpc_solver* h, Level& L) {
  HIPCHK(hipStreamSynchronize(h->stream));
  for (void* p : L.bd.owned) (void)hipFree(p);
  L.bd = BlockDense{};
  L.bdense = false;
}

// The row-product launch of step t of the block-dense form (forward, or backward with
// the transposed inverses): the blocks of the step as systems, or a single block.
static DenseTriDev bd_step(const Level& L, bool upper, int t) {
  const BlockDense& bd = L.bd;
  const std::vector<int>& step = upper ? bd.bstep : bd.fstep;
  const std::vector<int>& item = upper ? bd.bitem : bd.fitem;
  if (t < 0 || (size_t)t + 1 >= step.size() || item.size() != step.size())
    throw HipError{hipErrorInvalidValue, "block-dense form: inconsistent step tables"};
  DenseTriDev dt = bd.dt;
  dt.item_n = (upper ? bd.items_b : bd.items_f) + item[t];
  dt.nitem_n = item[t + 1] - item[t];
  dt.one_n = 0;
  dt.max_n = 0;
  for (int q = step[t]; q < step[t + 1]; ++q) dt.max_n = std::max(dt.max_n, bd.rows[upper ? bd.bblk[q] : q]);
  if (step[t + 1] - step[t] == 1) {  // one block: its rows and offsets need no table reads
    const int b = upper ? bd.bblk[step[t]] : step[t];
    dt.one_n = bd.rows[b];
    dt.one_voff = bd.start[b];
    dt.one_moff = bd.moff[b];
    dt.one_sys = b;
  }
  return dt;
}

static int bd_steps(const Level& L, bool upper) {
  return (int)(upper ? L.bd.bstep.size() : L.bd.fstep.size()) - 1;
}

// x = T^{-1} f (upper = false) or x = T^{-T} f (upper = true) through the block-dense
// form; g is a scratch vector of the level.
static void bdense_solve(cpc_solver* h, Level& L, bool upper, const void* f, void* x, void* g, const int* done) {
  const bool f32 = h->f32;
  const BlockDense& bd = L.bd;
  const DevCsr& off = upper ? bd.Uoff : bd.Loff;
  const std::vector<int>& rows = upper ? bd.brow : bd.frow;
  const int T = bd_steps(L, upper);
  for (int t = 0; t < T; ++t) {
    MatDev m = off.mat(f32);
    m.n = rows[t + 1] - rows[t];
    m.rp = off.rp + rows[t];
    m.rid = (upper ? bd.Urid : bd.Lrid) + rows[t];
    m.mask = mask_of(h, L.row_sys);
    spmv_or_throw(h, m, 1, x, f32, f, f32, g, f32, off.tpr, done);
    const DenseTriDev dt = dmask(h, bd_step(L, upper, t));
    if (upper) launch_dense_lower_t(h->stream, dt, f32, f32, g, x, done);
    else launch_dense_lower(h->stream, dt, f32, f32, g, x, done);
  }
}

// Rows per sweep block, level by level: the candidates' schedules are built and
// their forward and backward solves (and, on the finest level, the ILU(0) solves)
// timed on the level's own matrix; the fastest stays. A forced block size skips this.
static void tune_sweeps(cpc_solver* h) {
  if (h->opt.sweep_block_rows > 0 && h->opt.dense_smoother != 3) return;
  const bool f32 = h->f32;
  if (!h->opt.tune && h->opt.dense_smoother != 3) {
    // fixed rules (measured on the 1M-unknown pressure systems): the block-dense form
    // with 4096-row blocks between 8192 and 300000 smoothed rows
    for (size_t d = 0; d + 1 < h->lev.size(); ++d) {
      Level& L = h->lev[d];
      if (h->opt.dense_smoother == 1 || h->opt.dense_smoother == 2 || L.dense_smooth || L.sweep_rows <= 8192 ||
          L.sweep_rows > 300000)
        continue;
      const HostCsr sub = L.sweep_rows == L.A_host.n ? L.A_host : leading_rows(L.A_host, L.sweep_rows);
      if (build_blockdense(h, L, sub, 4096)) L.bdense = true;
      progress(h, "level " + std::to_string(d) + ": block-dense smoother, 4096-row blocks");
    }
    return;
  }
  for (size_t d = 0; d < h->lev.size(); ++d) {
    Level& L = h->lev[d];
    if (L.sweep_rows <= 4096) continue;
    const bool ilu = d == 0;
    const HostCsr sub = L.sweep_rows == L.A_host.n ? L.A_host : leading_rows(L.A_host, L.sweep_rows);
    void* f = d == 0 ? h->pin : L.f;
    void* u = d == 0 ? h->u1 : L.u;
    auto cost = [&] {
      return time_ms(h, 3, [&] {
        if (!L.dense_smooth) {
          run_sweep(h, SWEEP_LOWER, L.lower, L.fgs, f, u, nullptr, nullptr, nullptr);
          run_sweep(h, SWEEP_UPPER, L.upper, L.bgs, f, u, nullptr, nullptr, nullptr);
        }
        if (ilu && !h->iluk) {
          run_sweep(h, SWEEP_UNIT_LOWER, L.lower, h->ilu_l, h->res, h->y, nullptr, nullptr, nullptr);
          run_sweep(h, SWEEP_UPPER_OUT, L.upper, h->ilu_u, h->y, h->w, h->u1, h->u2, nullptr);
        }
      });
    };
    const bool try_r = L.sweep_rows <= 8000000 && !(L.dense_smooth && !ilu);
    const bool bd_ok = L.sweep_rows > 8192 && d + 1 < h->lev.size() && h->opt.dense_smoother == 0;
    auto gs_cost = [&] {
      return time_ms(h, 3, [&] {
        if (L.bdense) {
          bdense_solve(h, L, false, f, u, L.r, nullptr);
          bdense_solve(h, L, true, f, u, L.r, nullptr);
        } else if (L.dense_smooth) {
          launch_dense_lower(h->stream, L.dtri, f32, f32, f, u, nullptr);
          launch_dense_lower_t(h->stream, L.dtri, f32, f32, f, u, nullptr);
        } else {
          run_sweep(h, SWEEP_LOWER, L.lower, L.fgs, f, u, nullptr, nullptr, nullptr);
          run_sweep(h, SWEEP_UPPER, L.upper, L.bgs, f, u, nullptr, nullptr, nullptr);
        }
      });
    };
    // quick look: where block substitution already beats the sweeps by half, tuning the
    // sweeps' block size cannot change the outcome and is skipped (the block form stays
    // as the candidate to beat). Blocks of 4096 rows, or of 2048 / 1024 where the larger
    // inverses would not fit the form's memory bound or could not be read fast enough
    // to be that far ahead (batch levels of a million rows).
    std::map<int, float> bd_time;  // measured block-substitution candidates
    bool skip_r = false;
    const std::vector<int> lparts = (!L.parts.empty() && L.parts.front() == 0 && L.parts.back() == L.sweep_rows)
                                        ? L.parts
                                        : std::vector<int>{0, L.sweep_rows};
    // lower bound (ms) of one forward + backward block solve: its inverses read at the HBM peak
    const double ewidth = h->f32 ? 4.0 : 8.0;
    auto bd_floor = [&](int B) { return (float)(ewidth * blockdense_squares(lparts, B) / 8e12 * 1e3); };
    auto bd_mem = [&](int B) { return 16.0 * blockdense_squares(lparts, B); };
    int qB = 4096;
    const double cap = blockdense_cap();
    float ts = 0.f;
    if (try_r && bd_ok && !L.dense_smooth) {
      ts = gs_cost();
      // the look decides only when the form is 1.5x ahead: a block size whose inverses
      // alone take longer to read than ts / 1.5 cannot do that
      while (qB > 1024 && (bd_mem(qB) > cap || 1.5f * bd_floor(qB) >= ts)) qB /= 2;
    }
    if (try_r && bd_ok && !L.dense_smooth && qB < L.sweep_rows && bd_mem(qB) <= cap &&
        1.5f * bd_floor(qB) < ts) {
      progress(h, "level " + std::to_string(d) + ": block substitution with " + std::to_string(qB) + "-row blocks");
      if (build_blockdense(h, L, sub, qB)) {
        L.bdense = true;
        const float tb = gs_cost();
        bd_time[qB] = tb;
        if (tb * 1.5f < ts) skip_r = true;
        else free_blockdense(h, L);
      }
    }
    progress(h, "level " + std::to_string(d) + (skip_r ? ": block substitution well ahead, sweep block size kept"
                                                        : ": timing sweep block sizes"));
    float best = try_r && !skip_r ? cost() : 0.f;
    // build the sweeps with R rows per block (M segments per block in the one-wave form)
    // in a list of their own; keep them if they are faster, else restore the current ones
    auto try_build = [&](int R, int M) {
      DevSweepSched lo = L.lower, up = L.upper;
      SweepPackDev fg = L.fgs, bg = L.bgs, il = h->ilu_l, iu = h->ilu_u;
      const int oldR = L.sweep_R, oldM = L.wave_M;
      std::vector<void*> old;
      old.swap(L.sweep_owned);
      bool built = true;
      L.wave_M = M;
      const double tb0 = now_s();
      try {
        build_level_sweeps(h, L, sub, R, ilu);
      } catch (const HipError&) {
        built = false;  // the candidate does not fit the sweep kernel's LDS
        (void)hipGetLastError();
      }
      const double tb1 = now_s();
      const float t = built ? cost() : 0.f;
      if (built) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "level %zu: %d-row blocks, %d segments (%s): %.3f ms, built in %.2f s", d, R,
                      L.fgs.wave.ok ? L.fgs.wave.M : 1, L.fgs.wave.ok ? "one-wave" : "four-wave", t, tb1 - tb0);
        progress(h, buf);
      }
      if (built && t < best) {
        best = t;
        HIPCHK(hipStreamSynchronize(h->stream));
        for (void* p : old) (void)hipFree(p);
      } else {
        HIPCHK(hipStreamSynchronize(h->stream));
        for (void* p : L.sweep_owned) (void)hipFree(p);
        L.sweep_owned.swap(old);
        L.lower = lo;
        L.upper = up;
        L.fgs = fg;
        L.bgs = bg;
        h->ilu_l = il;
        h->ilu_u = iu;
        L.sweep_R = oldR;
        L.wave_M = oldM;
      }
    };
    if (try_r && !skip_r) {
      char buf[128];
      std::snprintf(buf, sizeof buf, "level %zu: %d-row blocks (%s): %.3f ms", d, L.sweep_R,
                    L.fgs.wave.ok ? "one-wave" : "four-wave", best);
      progress(h, buf);
    }
    // block sizes 64 .. 16384 (below 256 and above 8192: one-wave form only): 1024 and 4096 first,
    // then doubling and halving from the better of those for as long as each step
    // gains (the measured times fall and then rise with the block size, with noise that
    // a walk from a single start can stop on)
    std::set<int> tried{L.sweep_R};
    for (int R : {1024, 4096}) {
      if (!try_r || skip_r || tried.count(R) || R >= L.sweep_rows) continue;
      if (R > sweep_max_rows_per_block() && !L.fgs.wave.ok) continue;
      tried.insert(R);
      try_build(R, L.wave_M);
    }
    for (int dir = 0; dir < 2 && try_r && !skip_r; ++dir) {
      for (;;) {
        const int R = dir == 0 ? L.sweep_R * 2 : L.sweep_R / 2;
        if (R < 64 || R > 16384 || R >= L.sweep_rows || tried.count(R)) break;
        if ((R > sweep_max_rows_per_block() || R < 256) && !L.fgs.wave.ok) break;
        tried.insert(R);
        const int before = L.sweep_R;
        try_build(R, L.wave_M);
        if (L.sweep_R == before) break;
      }
    }
    // segments per block of the one-wave form at the chosen block size
    if (try_r && !skip_r && L.fgs.wave.ok && L.wave_stride > 0) {
      const int cur = L.fgs.wave.M;
      for (int M : {1, 2, 4})
        if (M != cur && L.sweep_R / M >= 256 && (M == 1 || L.wave_stride >= L.sweep_R / M))
          try_build(L.sweep_R, M);
      progress(h, "level " + std::to_string(d) + ": one-wave sweeps, " + std::to_string(L.sweep_R) +
                      "-row blocks in " + std::to_string(L.fgs.wave.M) + " segments");
    }
    // block-dense form of the Gauss-Seidel factor, blocks of 2048 / 4096 / 8192 rows
    if (h->opt.dense_smoother == 3 && d + 1 < h->lev.size()) {
      if (build_blockdense(h, L, sub, 2048)) L.bdense = true;  // forced form (tests)
      continue;
    }
    if (L.sweep_rows > 8192 && d + 1 < h->lev.size() && h->opt.dense_smoother != 1 &&
        h->opt.dense_smoother != 2) {
      float gbest = gs_cost();
      const bool was_dense = L.dense_smooth;
      // block substitution with B-row blocks; kept if faster than the best so far (the
      // current block-dense form, if any, is set aside meanwhile)
      auto try_bd = [&](int B) {
        Level keep;
        keep.bdense = L.bdense;
        std::swap(keep.bd, L.bd);
        L.bdense = false;
        bool better = false;
        progress(h, "level " + std::to_string(d) + ": block substitution with " + std::to_string(B) + "-row blocks");
        if (build_blockdense(h, L, sub, B)) {
          L.bdense = true;
          L.dense_smooth = false;
          const float t = gs_cost();
          bd_time[B] = t;
          L.dense_smooth = was_dense && !(t < gbest);
          better = t < gbest;
          if (better) gbest = t;
        }
        if (better) {
          HIPCHK(hipStreamSynchronize(h->stream));
          for (void* p : keep.bd.owned) (void)hipFree(p);
        } else {
          free_blockdense(h, L);
          L.bdense = keep.bdense;
          std::swap(keep.bd, L.bd);
        }
      };
      // block sizes from the middle out; 8192 only where the model t(B) = a / B + c B
      // fitted to the 2048 and 4096 timings predicts a gain, 1024 unless 4096 beat 2048
      // (in a batch, where each step takes a block of every system, the times do not
      // follow that model on the small side)
      for (int B : {4096, 2048, 8192, 1024}) {
        if (B >= L.sweep_rows) continue;
        if (L.bdense && L.bd.B == B) continue;  // kept from the quick look
        if (!(bd_floor(B) < gbest)) continue;   // reading its inverses alone takes longer
        if (bd_time.count(B) && !(bd_time[B] < gbest)) continue;  // timed in the quick look
        if (B == 1024 && bd_time.count(2048) && bd_time.count(4096) && bd_time[4096] < bd_time[2048]) continue;
        if (B == 8192 && bd_time.count(2048) && bd_time.count(4096)) {
          const double t2 = bd_time[2048], t4 = bd_time[4096];
          const double c = (2.0 * t4 - t2) / (2.0 * 4096.0 - 2048.0);  // from t2 = a/2048 + 2048c, t4 = a/4096 + 4096c
          const double a = (t2 - 2048.0 * c) * 2048.0;
          const double pred = a / B + c * B;
          if (!(pred < 0.97 * gbest)) continue;
        }
        try_bd(B);
      }
      // in a batch (many independent systems per step) small blocks can keep winning:
      // halve while the smallest size tried is the best
      for (int B = 512; B >= 256 && L.bdense && L.bd.B == 2 * B && bd_time.count(2 * B); B /= 2) try_bd(B);
      progress(h, "level " + std::to_string(d) + ": " +
                      (L.bdense ? "block-dense, " + std::to_string(L.bd.B) + "-row blocks"
                                : (L.dense_smooth ? std::string("explicit inverse") : "sweeps, " +
                                   std::to_string(L.sweep_R) + "-row blocks")));
      if (L.bdense && was_dense) {  // the block form replaces the whole-level inverse
        HIPCHK(hipStreamSynchronize(h->stream));
        for (void* p : L.dense_owned) (void)hipFree(p);
        L.dense_owned.clear();
        L.dtri = DenseTriDev{};
        L.dense_entries = 0.0;
        L.dense_smooth = false;
      }
    }
  }
  unsigned herr = 0;
  HIPCHK(hipMemcpy(&herr, h->sync.err, sizeof(unsigned), hipMemcpyDeviceToHost));
  if (herr) throw HipError{hipErrorUnknown, "a sweep wait exceeded its bound while tuning"};
}

// Concatenate the systems' hierarchies depth by depth and upload them. At depth d
// the level vector holds, in this order, the systems that are smoothed at d (still
// coarsened further) and then the systems whose coarsest level is d; matrices are
// block diagonal, so the leading smoothed rows couple only among themselves.
// Depth 0 keeps the callers' system order.
static int assemble_levels(cpc_solver* h, std::vector<SysHier>& sys, const cpc_options& o, std::string* msg) {
  const int ns = (int)sys.size();
  int D = 0;
  for (auto& S : sys) D = std::max(D, (int)S.A.size());
  // Depth 0 keeps the callers' order and smooths every system there: a system that is
  // its own coarsest level (one level, n <= max_coarse) gets empty rows in P, so no
  // coarse correction reaches it, and the exact solve A_0^{-1} f of the systems that
  // bottom out at depth 0 overwrites its rows at the end of the cycle (its V-cycle is
  // A_0^{-1}, as for a one-level hierarchy alone).
  const bool mixed0 = D > 1 && std::any_of(sys.begin(), sys.end(), [](const SysHier& S) { return S.A.size() < 2; });
  auto smoothed_at = [&](int d, int s) { return d + 1 < (int)sys[s].A.size() || (d == 0 && mixed0); };
  std::vector<std::vector<int>> order(D), off(D, std::vector<int>(ns, -1));
  std::vector<int> ntot(D, 0), nS(D, 0);
  for (int d = 0; d < D; ++d) {
    for (int s = 0; s < ns; ++s)
      if (smoothed_at(d, s)) order[d].push_back(s);
    const int nsm = (int)order[d].size();
    for (int s = 0; s < ns; ++s)
      if (d + 1 == (int)sys[s].A.size() && !smoothed_at(d, s)) order[d].push_back(s);
    int o_ = 0;
    for (int k = 0; k < (int)order[d].size(); ++k) {
      const int s = order[d][k];
      off[d][s] = o_;
      o_ += sys[s].A[d].n;
      if (k < nsm) nS[d] = o_;
    }
    ntot[d] = o_;
  }
  h->lev.assign(D, Level());
  h->lu_host.clear();
  for (int s = 0; s < ns; ++s) h->lu_host.insert(h->lu_host.end(), sys[s].lu.begin(), sys[s].lu.end());
  for (int d = 0; d < D; ++d) {
    Level& L = h->lev[d];
    progress(h, "level " + std::to_string(d) + ": " + std::to_string(ntot[d]) + " rows, " +
                    std::to_string(order[d].size()) + " systems");
    // block-diagonal matrix of depth d
    HostCsr& A = L.A_host;
    {
      std::vector<PlacedBlock> blk;
      for (int s : order[d]) blk.push_back({&sys[s].A[d], off[d][s], off[d][s]});
      place_blocks(blk, ntot[d], ntot[d], A);
    }
    L.nS = nS[d];
    upload_csr(h, A, L.A, true);
    L.nnzS = A.rp[L.nS];
    // prolongation from depth d+1 (rows: smoothed systems at d; columns: depth d+1 layout)
    if (d + 1 < D && L.nS > 0) {
      HostCsr& P = L.P_host;
      L.cf.clear();
      std::vector<PlacedBlock> pb, rb;
      std::vector<HostCsr> empty, tr;  // empty rows of one-level systems; per-system P^T
      empty.reserve(order[d].size());
      std::vector<int> with_p;
      for (int s : order[d]) {
        if (!smoothed_at(d, s)) continue;
        if (d + 1 >= (int)sys[s].A.size()) {  // one-level system at depth 0: empty rows
          HostCsr e;
          e.n = sys[s].A[d].n;
          e.rp.assign(e.n + 1, 0);
          empty.push_back(std::move(e));
          L.cf.insert(L.cf.end(), (size_t)sys[s].A[d].n, 0);
          continue;
        }
        with_p.push_back(s);
        L.cf.insert(L.cf.end(), sys[s].cf[d].begin(), sys[s].cf[d].end());
      }
      tr.resize(with_p.size());
      parallel_for((int)with_p.size(), setup_threads(), [&](int k) { tr[k] = transpose(sys[with_p[k]].P[d]); });
      size_t e = 0;
      for (int s : order[d]) {
        if (!smoothed_at(d, s)) continue;
        if (d + 1 >= (int)sys[s].A.size()) {
          pb.push_back({&empty[e++], off[d][s], 0});
          continue;
        }
        const size_t k = std::find(with_p.begin(), with_p.end(), s) - with_p.begin();
        pb.push_back({&sys[s].P[d], off[d][s], off[d + 1][s]});
        rb.push_back({&tr[k], off[d + 1][s], off[d][s]});
      }
      place_blocks(pb, L.nS, ntot[d + 1], P);
      HostCsr R;
      place_blocks(rb, ntot[d + 1], L.nS, R);
      upload_csr(h, P, L.P, false);
      upload_csr(h, R, L.R, false);
    }
    // exact solves of the systems that bottom out here
    {
      std::vector<int> doff, dn, dsys;
      std::vector<const std::vector<double>*> invs;
      for (int s : order[d])
        if (d + 1 == (int)sys[s].A.size()) {
          doff.push_back(off[d][s]);
          dn.push_back(sys[s].A[d].n);
          dsys.push_back(s);
          invs.push_back(&sys[s].inv);
        }
      L.dense = upload_dense_list(h, doff, dn, invs);
      L.dense_n = dn;
      if (h->batch && !dsys.empty()) L.dense.mask.of = dupload(dsys, h->owned, h->stream);
    }
    // batch system of every row of the level (per-system masks of the batched solve)
    if (h->batch) {
      std::vector<int> rs(ntot[d], -1);
      for (int s : order[d])
        std::fill(rs.begin() + off[d][s], rs.begin() + off[d][s] + sys[s].A[d].n, s);
      L.row_sys = dupload(rs, h->owned, h->stream);
    }
    // sweep schedules and packed rows: the smoothed rows (all rows at depth 0, for ILU(0))
    const int rows = (d == 0) ? ntot[0] : L.nS;
    L.parts.assign(1, 0);
    L.part_sys.clear();
    for (int s : order[d])
      if (off[d][s] + sys[s].A[d].n <= rows) {
        L.parts.push_back(off[d][s] + sys[s].A[d].n);
        L.part_sys.push_back(s);
      }
    if (rows > 0) {
      HostCsr sub = (rows == ntot[d]) ? A : leading_rows(A, rows);
      const int Rb = o.sweep_block_rows > 0 ? std::min(o.sweep_block_rows, sweep_max_rows_per_block())
                                            : choose_block_rows(rows);
      L.sweep_rows = rows;
      progress(h, "level " + std::to_string(d) + ": sweep forms");
      build_level_sweeps(h, L, sub, Rb, d == 0);
      upload_csr(h, strict_lower(sub), L.Ls, false);
      L.t = valloc(h, rows);
      if (L.nS > 0 && d + 1 < D) {
        progress(h, "level " + std::to_string(d) + ": dense forms");
        std::vector<int> dn, dv;
        for (int s : order[d])
          if (smoothed_at(d, s)) {
            dn.push_back(sys[s].A[d].n);
            dv.push_back(off[d][s]);
          }
        build_dense(h, L, dn, dv);
      }
      L.r = valloc(h, rows);
    }
    if (d > 0) {
      L.f = valloc(h, ntot[d]);
      L.u = valloc(h, ntot[d]);
    }
  }
  return CPC_OK;
}

// Vectors, device state and sweep counters of a handle whose levels are assembled.
static void allocate_work(cpc_solver* h) {
  const int n = h->n;
  h->lu = dupload(h->lu_host, h->owned, h->stream);
  if (h->f32) {
    h->lu32 = dalloc<float>(h->lu_host.size(), h->owned);
    launch_to_f32(h->stream, (int64_t)h->lu_host.size(), h->lu, h->lu32);
  }
  h->r = dalloc<double>(n, h->owned);
  h->z = dalloc<double>(n, h->owned);
  h->p = dalloc<double>(n, h->owned);
  h->q = dalloc<double>(n, h->owned);
  h->z64tmp = dalloc<double>(n, h->owned);
  h->pin = valloc(h, n);
  h->u1 = valloc(h, n);
  h->u2 = valloc(h, n);
  h->res = valloc(h, n);
  h->y = valloc(h, n);
  h->w = valloc(h, n);
  h->t = valloc(h, n);
  h->st = dalloc<PcgState>(1, h->owned);
  h->partials = dalloc<double>(kPartials, h->owned);
  h->sync.ticket = dalloc<unsigned>(1, h->owned);
  h->sync.exited = dalloc<unsigned>(1, h->owned);
  h->sync.err = dalloc<unsigned>(1, h->owned);
  for (void* v : {h->pin, h->u1, h->u2, h->res, h->y, h->w, h->t})
    HIPCHK(hipMemsetAsync(v, 0, esz_of(h) * (size_t)n, h->stream));
  for (void* v : {(void*)h->r, (void*)h->z, (void*)h->p, (void*)h->q, (void*)h->z64tmp})
    HIPCHK(hipMemsetAsync(v, 0, sizeof(double) * (size_t)n, h->stream));
  for (auto& L : h->lev) {
    for (void* v : {L.f, L.u})
      if (v) HIPCHK(hipMemsetAsync(v, 0, esz_of(h) * (size_t)L.A.n, h->stream));
    for (void* v : {L.r, L.t})
      if (v) HIPCHK(hipMemsetAsync(v, 0, esz_of(h) * (size_t)L.lower.d.n, h->stream));
  }
  HIPCHK(hipMemsetAsync(h->st, 0, sizeof(PcgState), h->stream));
  HIPCHK(hipMemsetAsync(h->sync.ticket, 0, sizeof(unsigned), h->stream));
  HIPCHK(hipMemsetAsync(h->sync.exited, 0, sizeof(unsigned), h->stream));
  HIPCHK(hipMemsetAsync(h->sync.err, 0, sizeof(unsigned), h->stream));
}

// Per-system scalars and chunk tables of a batch.
static void allocate_batch(cpc_solver* h) {
  const int ns = h->nsys;
  constexpr int kChunk = 2048;
  std::vector<int> chunk_sys, chunk_row, sys_chunk(ns + 1, 0);
  for (int s = 0; s < ns; ++s) {
    sys_chunk[s] = (int)chunk_sys.size();
    for (int r = 0; r < h->sys_n[s]; r += kChunk) {
      chunk_sys.push_back(s);
      chunk_row.push_back(h->sys_off[s] + r);
    }
  }
  sys_chunk[ns] = (int)chunk_sys.size();
  chunk_row.push_back(h->n);
  BatchDev& bd = h->bd;
  bd.nsys = ns;
  bd.nchunks = (int)chunk_sys.size();
  bd.chunk_sys = dupload(chunk_sys, h->owned, h->stream);
  bd.chunk_row = dupload(chunk_row, h->owned, h->stream);
  bd.sys_chunk = dupload(sys_chunk, h->owned, h->stream);
  bd.partials = dalloc<double>((size_t)4 * bd.nchunks, h->owned);
  bd.cnt = dalloc<unsigned>((size_t)4 * ns, h->owned);
  HIPCHK(hipMemsetAsync(bd.cnt, 0, sizeof(unsigned) * 4 * ns, h->stream));
  double** dv[] = {&bd.rz, &bd.pq, &bd.alpha, &bd.beta, &bd.rr, &bd.bb, &bd.relres};
  for (double** p : dv) {
    *p = dalloc<double>(ns, h->owned);
    HIPCHK(hipMemsetAsync(*p, 0, sizeof(double) * ns, h->stream));
  }
  bd.iters = dalloc<int>(ns, h->owned);
  bd.done = dalloc<int>(ns, h->owned);
  HIPCHK(hipMemsetAsync(bd.iters, 0, sizeof(int) * ns, h->stream));
  HIPCHK(hipMemsetAsync(bd.done, 0, sizeof(int) * ns, h->stream));
  h->btol = dalloc<double>(1, h->owned);
  h->bmaxit = dalloc<int>(1, h->owned);
  bd.tol_dev = h->btol;
  bd.maxit_dev = h->bmaxit;
}

static MatDev smoothed(const DevCsr& A, int nS, bool f32) {
  MatDev m = A.mat(f32);
  m.n = nS;
  return m;
}

static void vcycle(cpc_solver* h, int d, const void* f, void* u, const int* done) {
  Level& L = h->lev[d];
  const bool f32 = h->f32;
  if (L.nS > 0 && d + 1 < (int)h->lev.size()) {
    Level& C = h->lev[d + 1];
    const MatDev A = masked_rows(h, smoothed(L.A, L.nS, f32), L.row_sys);
    // (1) pre-smoothing from zero: u = (D+L)^{-1} f
    if (L.dense_smooth) launch_dense_lower(h->stream, dmask(h, L.dtri), f32, f32, f, u, done);
    else if (L.bdense) bdense_solve(h, L, false, f, u, L.r, done);
    else run_sweep(h, SWEEP_LOWER, L.lower, L.fgs, f, u, nullptr, nullptr, done);
    // (2a) f_c = R (f - A u)
    spmv_or_throw(h, A, 1, u, f32, f, f32, L.r, f32, L.A.tpr, done);
    spmv_or_throw(h, masked_rows(h, L.R.mat(f32), C.row_sys), 0, L.r, f32, nullptr, f32, C.f, f32, L.R.tpr, done);
    // (2b) coarse correction
    vcycle(h, d + 1, C.f, C.u, done);
    // (2c) u += P e
    spmv_or_throw(h, masked_rows(h, L.P.mat(f32), L.row_sys), 2, C.u, f32, nullptr, f32, u, f32, L.P.tpr, done);
    // (3) post-smoothing, one backward Gauss-Seidel sweep (S_l^T): the new u solves
    //     (D+U) u = f - L u_old, the strict lower part taken at the old values
    spmv_or_throw(h, masked_rows(h, L.Ls.mat(f32), L.row_sys), 1, u, f32, f, f32, L.t, f32, L.Ls.tpr, done);
    if (L.dense_smooth) launch_dense_lower_t(h->stream, dmask(h, L.dtri), f32, f32, L.t, u, done);  // T^{-T}
    else if (L.bdense) bdense_solve(h, L, true, L.t, u, L.r, done);
    else run_sweep(h, SWEEP_UPPER, L.upper, L.bgs, L.t, u, nullptr, nullptr, done);
  }
  // systems whose coarsest level is this one: e = A_0^{-1} f (FP64 inverse)
  if (L.dense.nblk > 0) launch_bdense(h->stream, lmask(h, L.dense), f, u, f32, done);
}

// z = (LU)^{-1} f (out = nullptr) or out = base + (LU)^{-1} f
static void ilu_apply(cpc_solver* h, const void* f, void* w, const void* base, void* out, const int* done) {
  run_sweep(h, SWEEP_UNIT_LOWER, ilu_lower_sched(h), h->ilu_l, f, h->y, nullptr, nullptr, done);
  run_sweep(h, out ? SWEEP_UPPER_OUT : SWEEP_UPPER, ilu_upper_sched(h), h->ilu_u, h->y, w, base, out, done);
}

// The V-cycle of the AMG(ILU(0)) comparator (Section 5): Algorithm 3.2 with ILU(0) as
// the smoother on the finest level, pre u = (LU)^{-1} f and post u += (LU)^{-1}(f - A u)
// (for symmetric A the ILU(0) product is symmetric up to rounding, so the factor is its
// own adjoint), and the Gauss-Seidel V-cycle below. Rows of systems solved exactly on
// the finest level (batches) are overwritten by that solve at the end.
static void vcycle_ilu_top(cpc_solver* h, const void* f, void* u, const int* done) {
  Level& L = h->lev[0];
  const bool f32 = h->f32;
  if (!(L.nS > 0 && h->lev.size() > 1)) {
    vcycle(h, 0, f, u, done);
    return;
  }
  Level& C = h->lev[1];
  const MatDev A = masked_rows(h, smoothed(L.A, L.nS, f32), L.row_sys);
  const MatDev R = masked_rows(h, L.R.mat(f32), C.row_sys), P = masked_rows(h, L.P.mat(f32), L.row_sys);
  ilu_apply(h, f, u, nullptr, nullptr, done);                                           // (1)
  spmv_or_throw(h, A, 1, u, f32, f, f32, L.r, f32, L.A.tpr, done);                       // (2a)
  spmv_or_throw(h, R, 0, L.r, f32, nullptr, f32, C.f, f32, L.R.tpr, done);
  vcycle(h, 1, C.f, C.u, done);                                                         // (2b)
  spmv_or_throw(h, P, 2, C.u, f32, nullptr, f32, u, f32, L.P.tpr, done);                 // (2c)
  spmv_or_throw(h, A, 1, u, f32, f, f32, L.t, f32, L.A.tpr, done);                       // (3)
  ilu_apply(h, L.t, L.r, nullptr, nullptr, done);
  launch_vec(h->stream, 1, L.nS, L.r, f32, nullptr, false, u, f32, done);
  if (L.dense.nblk > 0) launch_bdense(h->stream, lmask(h, L.dense), f, u, f32, done);
}

// res = r - A u with FP64 A and FP64 r (outer residual of Algorithm 2.1)
static void outer_residual(cpc_solver* h, const double* r, const void* u, void* res, const int* done) {
  Level& L = h->lev[0];
  spmv_or_throw(h, masked_rows(h, L.A.mat(false), L.row_sys), 1, u, h->f32, r, false, res, h->f32, L.A.tpr,
                done);
}

static void apply_op(cpc_solver* h, int op, const double* r, double* z, const int* done) {
  const bool f32 = h->f32;
  const int n = h->n;
  const void* rin = r;
  if (f32 && op != CPC_OP_NONE) {
    launch_vec(h->stream, 2, n, r, false, nullptr, false, h->pin, true, done);
    rin = h->pin;
  }
  switch (op) {
    case CPC_OP_COMBINED: {
      if (!h->opt.swap_roles) {
        vcycle(h, 0, rin, h->u1, done);                        // (1) u1 = S r
        outer_residual(h, r, h->u1, h->res, done);             //     r - A u1
        ilu_apply(h, h->res, h->w, h->u1, h->u2, done);        // (2) u2 = u1 + B (r - A u1)
        outer_residual(h, r, h->u2, h->res, done);             //     r - A u2
        vcycle(h, 0, h->res, h->t, done);                      // (3) S^T (r - A u2), S^T = S
        launch_vec(h->stream, 0, n, h->u2, f32, h->t, f32, z, false, done);
      } else {
        ilu_apply(h, rin, h->u1, nullptr, nullptr, done);      // (1) u1 = S r, S = ILU(0)
        outer_residual(h, r, h->u1, h->res, done);
        vcycle(h, 0, h->res, h->t, done);                      // (2) u2 = u1 + V (r - A u1)
        launch_vec(h->stream, 0, n, h->u1, f32, h->t, f32, h->u2, f32, done);
        outer_residual(h, r, h->u2, h->res, done);
        ilu_apply(h, h->res, h->t, nullptr, nullptr, done);   // (3) ILU^T = ILU for symmetric A
        launch_vec(h->stream, 0, n, h->u2, f32, h->t, f32, z, false, done);
      }
      break;
    }
    case CPC_OP_AMG: {
      vcycle(h, 0, rin, h->u1, done);
      outer_residual(h, r, h->u1, h->res, done);
      vcycle(h, 0, h->res, h->t, done);
      launch_vec(h->stream, 0, n, h->u1, f32, h->t, f32, z, false, done);
      break;
    }
    case CPC_OP_AMG_ILU: {  // two ILU(0)-smoothed cycles: z = V'(r) + V'(r - A V'(r))
      vcycle_ilu_top(h, rin, h->u1, done);
      outer_residual(h, r, h->u1, h->res, done);
      vcycle_ilu_top(h, h->res, h->t, done);
      launch_vec(h->stream, 0, n, h->u1, f32, h->t, f32, z, false, done);
      break;
    }
    case CPC_OP_BBAR: {
      // I - B-bar A = (I - BA)(I - S~A)(I - BA) from a zero start, the propagators
      // acting right to left: u1 = B r, u2 = u1 + S~(r - A u1), z = u2 + B(r - A u2),
      // with S~(g) = a + V(g - A a), a = V(g), i.e. u2 = (u1 + a) + V(r - A(u1 + a))
      ilu_apply(h, rin, h->u1, nullptr, nullptr, done);
      outer_residual(h, r, h->u1, h->res, done);
      vcycle(h, 0, h->res, h->t, done);
      launch_vec(h->stream, 0, n, h->u1, f32, h->t, f32, h->u2, f32, done);
      outer_residual(h, r, h->u2, h->res, done);
      vcycle(h, 0, h->res, h->t, done);
      launch_vec(h->stream, 1, n, h->t, f32, nullptr, false, h->u2, f32, done);
      outer_residual(h, r, h->u2, h->res, done);
      ilu_apply(h, h->res, h->t, nullptr, nullptr, done);
      launch_vec(h->stream, 0, n, h->u2, f32, h->t, f32, z, false, done);
      break;
    }
    case CPC_OP_ILU: {
      ilu_apply(h, rin, h->u1, nullptr, nullptr, done);
      launch_vec(h->stream, 2, n, h->u1, f32, nullptr, false, z, false, done);
      break;
    }
    case CPC_OP_ADDITIVE: {
      vcycle(h, 0, rin, h->u1, done);
      outer_residual(h, r, h->u1, h->res, done);
      vcycle(h, 0, h->res, h->t, done);
      launch_vec(h->stream, 0, n, h->u1, f32, h->t, f32, h->z64tmp, false, done);  // S~ r
      ilu_apply(h, rin, h->u2, nullptr, nullptr, done);                           // B r
      launch_vec(h->stream, 0, n, h->z64tmp, false, h->u2, f32, z, false, done);
      break;
    }
    case CPC_OP_VCYCLE: {
      vcycle(h, 0, rin, h->u1, done);
      launch_vec(h->stream, 2, n, h->u1, f32, nullptr, false, z, false, done);
      break;
    }
    case CPC_OP_FGS:
    case CPC_OP_BGS: {
      Level& L = h->lev[0];
      // (D+L)^{-1} f and (D+U)^{-1} f: one forward or backward sweep from a zero start
      if (L.dense_smooth) {
        if (op == CPC_OP_FGS) launch_dense_lower(h->stream, L.dtri, f32, f32, rin, h->u1, done);
        else launch_dense_lower_t(h->stream, L.dtri, f32, f32, rin, h->u1, done);
      } else if (L.bdense) {
        bdense_solve(h, L, op == CPC_OP_BGS, rin, h->u1, L.r, done);
      } else if (op == CPC_OP_FGS) {
        run_sweep(h, SWEEP_LOWER, L.lower, L.fgs, rin, h->u1, nullptr, nullptr, done);
      } else {
        run_sweep(h, SWEEP_UPPER, L.upper, L.bgs, rin, h->u1, nullptr, nullptr, done);
      }
      launch_vec(h->stream, 2, n, h->u1, f32, nullptr, false, z, false, done);
      break;
    }
    default:
      launch_vec(h->stream, 2, n, r, false, nullptr, false, z, false, done);
      break;
  }
}

static int prec_to_op(int prec) {
  switch (prec) {
    case CPC_PREC_COMBINED: return CPC_OP_COMBINED;
    case CPC_PREC_AMG: return CPC_OP_AMG;
    case CPC_PREC_ILU: return CPC_OP_ILU;
    case CPC_PREC_ADDITIVE: return CPC_OP_ADDITIVE;
    case CPC_PREC_AMG_ILU: return CPC_OP_AMG_ILU;
    case CPC_PREC_BBAR: return CPC_OP_BBAR;
    default: return CPC_OP_NONE;
  }
}

static MatDev pcg_operator(const cpc_solver* h) {
  MatDev m = h->lev[0].A.mat(false);
  if (h->op_vals) m.v = h->op_vals;
  return m;
}

static void enqueue_iteration(cpc_solver* h, int prec, double* x) {
  int* done = &h->st->done;
  const DevCsr& A = h->lev[0].A;
  launch_spmv_pq(h->stream, pcg_operator(h), h->p, h->q, h->partials, h->st, A.tpr);
  launch_update_xr(h->stream, h->n, x, h->r, h->p, h->q, h->partials, h->st);
  apply_op(h, prec_to_op(prec), h->r, h->z, done);
  launch_dot_rz(h->stream, h->n, h->r, h->z, h->p, h->partials, h->st, false);
  launch_update_p(h->stream, h->n, h->z, h->p, h->st);
}

// Algorithmic HBM bytes of one application of each piece (byte model of the
// measurement plan: matrix streams read once per pass, vectors once per kernel).
// Bytes of the smoothing on level d of one V-cycle: pre-smoothing, the strict-lower
// pass of the post-smoothing and the post-smoothing (same model as vcycle_bytes).
static double level_smooth_bytes(const cpc_solver* h, size_t d) {
  const double vb = h->f32 ? 4.0 : 8.0;
  const double mb = h->f32 ? 8.0 : 12.0;
  const Level& L = h->lev[d];
  if (!(L.nS > 0 && d + 1 < h->lev.size())) return 0.0;
  const double nz = (double)L.nnzS, n = L.nS, half = 0.5 * (nz - n);
  const double eb = h->f32 ? 4.0 : 8.0;
  double one;
  if (L.bdense) one = eb * L.bd.entries + (double)L.bd.Loff.nnz * mb + 4.0 * n + 3.0 * vb * n;
  else if (L.dense_smooth) one = eb * L.dense_entries + 2.0 * vb * n;
  else one = vb * n + (half + n) * mb + 4.0 * n + 2.0 * vb * n;
  return 2.0 * one + half * mb + 4.0 * n + 3.0 * vb * n;
}

static double vcycle_bytes(const cpc_solver* h) {
  const double vb = h->f32 ? 4.0 : 8.0;           // vector element
  const double mb = h->f32 ? 8.0 : 12.0;          // matrix entry (value + column)
  double b = 0.0;
  for (size_t d = 0; d < h->lev.size(); ++d) {
    const Level& L = h->lev[d];
    if (L.nS > 0 && d + 1 < h->lev.size()) {
      const double nz = (double)L.nnzS, n = L.nS, nc = h->lev[d + 1].A.n;
      const double p = (double)L.P.nnz;
      const double half = 0.5 * (nz - n);
      const double eb = h->f32 ? 4.0 : 8.0;  // explicit inverse entry
      const double bdb = eb * L.bd.entries + (double)L.bd.Loff.nnz * mb + 4.0 * n + 3.0 * vb * n;
      if (L.bdense) b += bdb;                                     // block-dense T^{-1} f
      else if (L.dense_smooth) b += eb * L.dense_entries + 2.0 * vb * n;    // T^{-1} f
      else b += vb * n + (half + n) * mb + 4.0 * n + 2.0 * vb * n;  // marker fill + forward GS from zero
      b += nz * mb + 4.0 * n + 3.0 * vb * n;                   // residual
      b += p * mb + 4.0 * nc + vb * n + vb * nc;               // restriction
      b += p * mb + 4.0 * n + 2.0 * vb * n + vb * nc;          // prolongation + correction
      b += half * mb + 4.0 * n + 3.0 * vb * n;                 // f - L u (old values)
      if (L.bdense) b += bdb;                                     // block-dense T^{-T} (f - L u)
      else if (L.dense_smooth) b += eb * L.dense_entries + 2.0 * vb * n;    // T^{-T} (f - L u)
      else b += vb * n + (half + n) * mb + 4.0 * n + 2.0 * vb * n;  // marker fill + (D+U) solve
    }
    for (int n0 : L.dense_n) b += 8.0 * n0 * n0 + 2.0 * vb * n0;  // exact coarsest solves
  }
  return b;
}

// Bytes of one launch of a kernel family on level d (same model as vcycle_bytes).
static double kernel_bytes(const cpc_solver* h, int kernel, int d) {
  const double vb = h->f32 ? 4.0 : 8.0;
  const double mb = h->f32 ? 8.0 : 12.0;
  const Level& L = h->lev[d];
  const bool fine = (kernel == CPC_K_SPMV_PQ || kernel == CPC_K_ILU_L || kernel == CPC_K_ILU_U);
  const double nz = fine ? (double)L.A.nnz : (double)L.nnzS, n = fine ? (double)L.A.n : (double)L.nS;
  const double half = 0.5 * (nz - n);
  const double nc = (d + 1 < (int)h->lev.size()) ? (double)h->lev[d + 1].A.n : 0.0;
  const double p = (double)L.P.nnz;
  switch (kernel) {
    case CPC_K_SPMV_PQ: return 12.0 * nz + 4.0 * n + 16.0 * n;
    case CPC_K_FGS:
    case CPC_K_BGS:
      if (L.bdense)
        return (h->f32 ? 4.0 : 8.0) * L.bd.entries + (double)L.bd.Loff.nnz * mb + 4.0 * n + 3.0 * vb * n;
      if (L.dense_smooth) return (h->f32 ? 4.0 : 8.0) * L.dense_entries + 2.0 * vb * n;
      return (half + n) * mb + 4.0 * n + 2.0 * vb * n;
    case CPC_K_ILU_L: return half * mb + 4.0 * n + 2.0 * vb * n;
    case CPC_K_ILU_U: return (half + n) * mb + 4.0 * n + 4.0 * vb * n;
    case CPC_K_RESIDUAL: return nz * mb + 4.0 * n + 3.0 * vb * n;
    case CPC_K_RESTRICT: return p * mb + 4.0 * nc + vb * n + vb * nc;
    case CPC_K_PROLONG: return p * mb + 4.0 * n + 2.0 * vb * n + vb * nc;
    default: return 0.0;
  }
}

static double prec_bytes(const cpc_solver* h, int prec) {
  const double vb = h->f32 ? 4.0 : 8.0;
  const double mb = h->f32 ? 8.0 : 12.0;
  const double nz = (double)h->lev[0].A.nnz, n = h->n;
  const double half = 0.5 * (nz - n);
  const double ilo = h->iluk ? h->ilu_lnnz : half, iup = h->iluk ? h->ilu_unnz : half + n;
  const double ilu = (ilo * mb + 4.0 * n + 2.0 * vb * n) + (iup * mb + 4.0 * n + 4.0 * vb * n) +
                     2.0 * vb * n;  // L and U solves, marker fills
  const double outer = nz * 12.0 + 4.0 * n + 8.0 * n + 2.0 * vb * n;
  const double V = vcycle_bytes(h);
  const double conv = h->f32 ? 12.0 * n : 0.0;
  switch (prec) {
    case CPC_PREC_COMBINED: return conv + 2.0 * V + ilu + 2.0 * outer + (2.0 * vb + 8.0) * n;
    case CPC_PREC_AMG: return conv + 2.0 * V + outer + (2.0 * vb + 8.0) * n;
    case CPC_PREC_ILU: return conv + ilu + (vb + 8.0) * n;
    case CPC_PREC_ADDITIVE: return conv + 2.0 * V + outer + ilu + 2.0 * (2.0 * vb + 8.0) * n;
    case CPC_PREC_AMG_ILU: {
      // each cycle trades the finest level's two sweeps (and the strict-lower pass)
      // for two ILU(0) applications, a residual and an axpy
      const double Vi = V - level_smooth_bytes(h, 0) + 2.0 * ilu + (nz * mb + 4.0 * n + 3.0 * vb * n) +
                        3.0 * vb * n;
      return conv + 2.0 * Vi + outer + (2.0 * vb + 8.0) * n;
    }
    case CPC_PREC_BBAR: return conv + 2.0 * V + 2.0 * ilu + 3.0 * outer + 3.0 * (2.0 * vb + 8.0) * n;
    default: return 16.0 * n;
  }
}

static double iteration_bytes(const cpc_solver* h, int prec) {
  const double nz = (double)h->lev[0].A.nnz, n = h->n;
  const double pcg = (12.0 * nz + 4.0 * n + 16.0 * n) + 48.0 * n + 16.0 * n + 24.0 * n;
  return pcg + prec_bytes(h, prec);
}

// ---------------------------------------------------------------------------
// Method bytes: what the method itself must move, whatever form evaluates a step.
// Every matrix stream is read once per pass the algorithm makes over it (an entry is
// its value and its 4-byte column, a row its 4-byte pointer) and every vector is read
// or written once per step. A natural-order Gauss-Seidel sweep from zero reads the
// lower triangle with the diagonal; the in-place backward sweep reads whole rows and
// the old and new values; ILU(0)'s triangular solves read L (strictly lower) and U
// (upper with the diagonal). FP32 preconditioner data: 4-byte values and vectors.
// These do not depend on how a sweep is evaluated (level-scheduled, block
// substitution or explicit inverse), so they rate every form against one yardstick.
struct MethodUnits {
  double E;  // bytes of one matrix entry of the preconditioner (value + column)
  double V;  // bytes of one preconditioner vector element
};

static MethodUnits method_units(const cpc_solver* h) {
  return h->f32 ? MethodUnits{8.0, 4.0} : MethodUnits{12.0, 8.0};
}

// forward Gauss-Seidel from zero on n rows, nz entries: lower triangle + diagonal,
// row pointers, f read, x written
static double m_fgs(const MethodUnits& u, double nz, double n) { return u.E * 0.5 * (nz + n) + 4.0 * n + 2.0 * u.V * n; }
// backward Gauss-Seidel in place: whole rows, f read, old x read, new x written
static double m_bgs(const MethodUnits& u, double nz, double n) { return u.E * nz + 4.0 * n + 3.0 * u.V * n; }
// residual f - A u on the level: whole rows, u and f read, r written
static double m_res(const MethodUnits& u, double nz, double n) { return u.E * nz + 4.0 * n + 3.0 * u.V * n; }
// f_c = R r (R = P^T with p entries, nc rows) and u += P e
static double m_restrict(const MethodUnits& u, double p, double n, double nc) {
  return u.E * p + 4.0 * nc + u.V * n + u.V * nc;
}
static double m_prolong(const MethodUnits& u, double p, double n, double nc) {
  return u.E * p + 4.0 * n + 2.0 * u.V * n + u.V * nc;
}

// one V-cycle (Algorithm 3.2) over the whole hierarchy
static double method_vcycle_bytes(const cpc_solver* h) {
  const MethodUnits u = method_units(h);
  double b = 0.0;
  for (size_t d = 0; d < h->lev.size(); ++d) {
    const Level& L = h->lev[d];
    if (L.nS > 0 && d + 1 < h->lev.size()) {
      const double nz = (double)L.nnzS, n = L.nS, nc = h->lev[d + 1].A.n, p = (double)L.P.nnz;
      b += m_fgs(u, nz, n) + m_res(u, nz, n) + m_restrict(u, p, n, nc) + m_prolong(u, p, n, nc) + m_bgs(u, nz, n);
    }
    for (int n0 : L.dense_n) b += 8.0 * n0 * n0 + 2.0 * u.V * n0;  // exact coarsest solve
  }
  return b;
}

// ILU solves: L strictly lower (unit diagonal implied), U with the diagonal; `axpy`:
// the U-solve also reads u1 and writes u2 = u1 + w (step 2 of Algorithm 2.1)
static double method_ilu_bytes(const cpc_solver* h, bool axpy) {
  const MethodUnits u = method_units(h);
  const double nz = (double)h->lev[0].A.nnz, n = h->n;
  const double lo = h->iluk ? h->ilu_lnnz : 0.5 * (nz - n), up = h->iluk ? h->ilu_unnz : 0.5 * (nz + n);
  return (u.E * lo + 4.0 * n + 2.0 * u.V * n) + (u.E * up + 4.0 * n + (axpy ? 3.0 : 2.0) * u.V * n);
}

static double method_prec_bytes(const cpc_solver* h, int prec) {
  const MethodUnits u = method_units(h);
  const double nz = (double)h->lev[0].A.nnz, n = h->n;
  const double outer = 12.0 * nz + 4.0 * n + 8.0 * n + 2.0 * u.V * n;  // FP64 r - A u
  const double add = (2.0 * u.V + 8.0) * n;                             // z = a + b
  const double V = method_vcycle_bytes(h);
  switch (prec) {
    case CPC_PREC_COMBINED: return V + outer + method_ilu_bytes(h, true) + outer + V + add;
    case CPC_PREC_AMG: return V + outer + V + add;
    case CPC_PREC_ILU: return method_ilu_bytes(h, false);
    case CPC_PREC_ADDITIVE: return 2.0 * V + outer + add + method_ilu_bytes(h, false) + add;
    case CPC_PREC_AMG_ILU: {
      // the finest level's Gauss-Seidel pair of each cycle becomes ILU(0) before and after
      // the coarse correction (post: residual, ILU solves, u += w)
      const Level& L0 = h->lev[0];
      double fine_gs = 0.0;
      if (L0.nS > 0 && h->lev.size() > 1) fine_gs = m_fgs(u, (double)L0.nnzS, L0.nS) + m_bgs(u, (double)L0.nnzS, L0.nS);
      const double Vi = V - fine_gs + 2.0 * method_ilu_bytes(h, false) + m_res(u, nz, n) + 3.0 * u.V * n;
      return Vi + outer + Vi + add;
    }
    case CPC_PREC_BBAR:
      return method_ilu_bytes(h, false) + outer + V + add + outer + V + add + outer + method_ilu_bytes(h, false) + add;
    default: return 16.0 * n;
  }
}

// PCG's own steps (FP64): q = A p with <p,q>, x and r updates with ||r||^2, <r,z>, p update
static double method_pcg_bytes(const cpc_solver* h) {
  const double nz = (double)h->lev[0].A.nnz, n = h->n;
  return (12.0 * nz + 4.0 * n + 16.0 * n) + 48.0 * n + 16.0 * n + 24.0 * n;
}

static double method_iteration_bytes(const cpc_solver* h, int prec) {
  return method_pcg_bytes(h) + method_prec_bytes(h, prec);
}

// before the first iteration: r = b - A x0 (or r = b), z = B r, <r,z>, p = z
static double method_initial_bytes(const cpc_solver* h, int prec) {
  const double nz = (double)h->lev[0].A.nnz, n = h->n;
  return (12.0 * nz + 28.0 * n) + method_prec_bytes(h, prec) + 16.0 * n + 16.0 * n;
}

// Method bytes of one launch of a kernel family on level d (the §(d)-style per-kernel
// figures; the backward Gauss-Seidel family is the triangular (D+U) solve, the strict
// lower pass over the old values being a separate SpMV).
static double method_kernel_bytes(const cpc_solver* h, int kernel, int d) {
  const MethodUnits u = method_units(h);
  const Level& L = h->lev[d];
  const bool fine = (kernel == CPC_K_SPMV_PQ || kernel == CPC_K_ILU_L || kernel == CPC_K_ILU_U);
  const double nz = fine ? (double)L.A.nnz : (double)L.nnzS, n = fine ? (double)L.A.n : (double)L.nS;
  const double nc = (d + 1 < (int)h->lev.size()) ? (double)h->lev[d + 1].A.n : 0.0;
  const double p = (double)L.P.nnz;
  const double lo = h->iluk ? h->ilu_lnnz : 0.5 * (nz - n), up = h->iluk ? h->ilu_unnz : 0.5 * (nz + n);
  switch (kernel) {
    case CPC_K_SPMV_PQ: return 12.0 * nz + 20.0 * n;
    case CPC_K_FGS: return m_fgs(u, nz, n);
    case CPC_K_BGS: return m_fgs(u, nz, n);  // (D+U) solve: upper triangle + diagonal, t read, u written
    case CPC_K_ILU_L: return u.E * lo + 4.0 * n + 2.0 * u.V * n;
    case CPC_K_ILU_U: return u.E * up + 4.0 * n + 3.0 * u.V * n;
    case CPC_K_RESIDUAL: return m_res(u, nz, n);
    case CPC_K_RESTRICT: return m_restrict(u, p, n, nc);
    case CPC_K_PROLONG: return m_prolong(u, p, n, nc);
    default: return 0.0;
  }
}

static cpc_status run_solve(cpc_solver* h, int prec, const double* b, double* x, int use_x0, double tol, int maxit,
                            int32_t* iters, double* relres, bool eager = false) {
  if (!h) return set_err(CPC_E_ARG, "null handle");
  if (h->batch) return set_err(CPC_E_ARG, "batch handle: use cpc_solve_batch");
  if (!b || !x) return set_err(CPC_E_ARG, "null vector");
  if (maxit < 0 || !(tol >= 0.0)) return set_err(CPC_E_ARG, "maxit must be >= 0 and tol >= 0");
  if (prec < 0 || prec >= kNumPrec) return set_err(CPC_E_ARG, "unknown preconditioner");
  const double t0 = now_s();
  try {
    PcgState init{};
    init.tol = tol;
    init.maxit = maxit;
    HIPCHK(hipMemcpyAsync(h->st, &init, sizeof(init), hipMemcpyHostToDevice, h->stream));
    const DevCsr& A = h->lev[0].A;
    launch_pcg_init(h->stream, pcg_operator(h), b, x, h->r, use_x0, h->partials, h->st, A.tpr);
    apply_op(h, prec_to_op(prec), h->r, h->z, &h->st->done);
    launch_dot_rz(h->stream, h->n, h->r, h->z, h->p, h->partials, h->st, true);
    HIPCHK(hipGetLastError());
    PcgState hs{};
    HIPCHK(hipMemcpyAsync(&hs, h->st, sizeof(hs), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    const int every = h->opt.check_every;
    bool use_graph = h->opt.use_graph != 0 && !eager;
    if (use_graph && (!h->graph[prec] || h->graph_x[prec] != x)) {
      if (h->graph[prec]) {
        (void)hipGraphExecDestroy(h->graph[prec]);
        (void)hipGraphDestroy(h->graph_src[prec]);
        h->graph[prec] = nullptr;
        h->graph_src[prec] = nullptr;
      }
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      try {
        enqueue_iteration(h, prec, x);
      } catch (...) {
        (void)hipStreamEndCapture(h->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      HIPCHK(hipStreamEndCapture(h->stream, &g));
      hipGraphExec_t ge = nullptr;
      hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        throw HipError{e, "hipGraphInstantiate"};
      }
      h->graph_src[prec] = g;
      h->graph[prec] = ge;
      h->graph_x[prec] = x;
    }
    int launched = 0;
    const int it0 = hs.iters;
    const double rel0 = hs.relres;
    while (!hs.done && launched < maxit) {
      const int k = std::min(every > 0 ? every : predicted_chunk(hs, it0, rel0), maxit - launched);
      for (int i = 0; i < k; ++i) {
        if (use_graph) HIPCHK(hipGraphLaunch(h->graph[prec], h->stream));
        else enqueue_iteration(h, prec, x);
      }
      launched += k;
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(&hs, h->st, sizeof(hs), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    unsigned herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, h->sync.err, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (hs.done == DONE_ZERO_RHS) {
      launch_vec(h->stream, 3, h->n, nullptr, false, nullptr, false, x, false, nullptr);
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    h->stats.iters = hs.iters;
    h->stats.relres = hs.relres;
    h->stats.solve_s = now_s() - t0;
    h->stats.bytes_per_iter = iteration_bytes(h, prec);
    h->stats.bytes_initial = (12.0 * h->lev[0].A.nnz + 40.0 * h->n) + prec_bytes(h, prec) + 24.0 * h->n;
    h->stats.method_bytes_per_iter = method_iteration_bytes(h, prec);
    h->stats.method_bytes_initial = method_initial_bytes(h, prec);
    if (iters) *iters = hs.iters;
    if (relres) *relres = hs.relres;
    cpc_status status = CPC_OK;
    if (herr) {
      HIPCHK(hipMemsetAsync(h->sync.err, 0, sizeof(unsigned), h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      status = set_err(CPC_E_DEVICE, "a sweep wait exceeded its bound");
    } else if (hs.done == DONE_BREAKDOWN) {
      status = set_err(CPC_E_BREAKDOWN, "PCG breakdown (<p,Ap> <= 0, <r,z> <= 0 or non-finite value)");
    } else if (hs.done == DONE_CONVERGED || hs.done == DONE_ZERO_RHS) {
      status = CPC_OK;
    } else {
      status = set_err(CPC_E_MAXIT, "no convergence within maxit");
    }
    h->stats.status = status;
    return status;
  } catch (const HipError& e) {
    return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
}

static void enqueue_batch_iteration(cpc_solver* h, int prec, double* x) {
  const DevCsr& A = h->lev[0].A;
  launch_bspmv_pq(h->stream, h->bd, A.mat(false), h->p, h->q, A.tpr);
  launch_bupdate_xr(h->stream, h->bd, x, h->r, h->p, h->q);
  apply_op(h, prec_to_op(prec), h->r, h->z, nullptr);
  launch_bdot_rz(h->stream, h->bd, h->r, h->z, h->p, false);
  launch_bupdate_p(h->stream, h->bd, h->z, h->p);
}

static cpc_status run_solve_batch(cpc_solver* h, int prec, const double* b, double* x, double tol, int maxit,
                                  int32_t* iters, double* relres) {
  if (!h || !h->batch) return set_err(CPC_E_ARG, "not a batch handle");
  if (!b || !x) return set_err(CPC_E_ARG, "null vector");
  if (maxit < 0 || !(tol >= 0.0)) return set_err(CPC_E_ARG, "maxit must be >= 0 and tol >= 0");
  const double t0 = now_s();
  const int ns = h->nsys;
  // the preconditioner's launches of this solve skip systems that have stopped
  struct MaskScope {
    cpc_solver* h;
    ~MaskScope() { h->mask_done = nullptr; }
  } mask_scope{h};
  h->mask_done = h->bd.done;
  try {
    HIPCHK(hipMemcpyAsync(h->btol, &tol, sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->bmaxit, &maxit, sizeof(int), hipMemcpyHostToDevice, h->stream));
    launch_binit(h->stream, h->bd, b, x, h->r);
    apply_op(h, prec_to_op(prec), h->r, h->z, nullptr);
    launch_bdot_rz(h->stream, h->bd, h->r, h->z, h->p, true);
    HIPCHK(hipGetLastError());
    std::vector<int> done(ns, 0);
    HIPCHK(hipMemcpyAsync(done.data(), h->bd.done, sizeof(int) * ns, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    auto all_done = [&]() {
      for (int v : done)
        if (!v) return false;
      return true;
    };
    const bool use_graph = h->opt.use_graph != 0;
    if (use_graph && (!h->bgraph[prec] || h->bgraph_x[prec] != x)) {
      if (h->bgraph[prec]) {
        (void)hipGraphExecDestroy(h->bgraph[prec]);
        (void)hipGraphDestroy(h->bgraph_src[prec]);
        h->bgraph[prec] = nullptr;
        h->bgraph_src[prec] = nullptr;
      }
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      try {
        enqueue_batch_iteration(h, prec, x);
      } catch (...) {
        (void)hipStreamEndCapture(h->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      HIPCHK(hipStreamEndCapture(h->stream, &g));
      hipGraphExec_t ge = nullptr;
      hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        throw HipError{e, "hipGraphInstantiate"};
      }
      h->bgraph_src[prec] = g;
      h->bgraph[prec] = ge;
      h->bgraph_x[prec] = x;
    }
    const int every = std::max(1, (int)h->opt.check_every);  // batch: every iteration unless set
    int launched = 0;
    while (!all_done() && launched < maxit) {
      const int k = std::min(every, maxit - launched);
      for (int i = 0; i < k; ++i) {
        if (use_graph) HIPCHK(hipGraphLaunch(h->bgraph[prec], h->stream));
        else enqueue_batch_iteration(h, prec, x);
      }
      launched += k;
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(done.data(), h->bd.done, sizeof(int) * ns, hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    std::vector<int> it(ns);
    std::vector<double> rel(ns);
    unsigned herr = 0;
    HIPCHK(hipMemcpyAsync(it.data(), h->bd.iters, sizeof(int) * ns, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(rel.data(), h->bd.relres, sizeof(double) * ns, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(done.data(), h->bd.done, sizeof(int) * ns, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(&herr, h->sync.err, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    int maxits = 0;
    for (int s = 0; s < ns; ++s) {
      if (iters) iters[s] = it[s];
      if (relres) relres[s] = rel[s];
      maxits = std::max(maxits, it[s]);
    }
    h->stats.iters = maxits;
    h->stats.solve_s = now_s() - t0;
    h->stats.bytes_per_iter = iteration_bytes(h, prec);
    h->stats.bytes_initial = (12.0 * h->lev[0].A.nnz + 40.0 * h->n) + prec_bytes(h, prec) + 24.0 * h->n;
    h->stats.method_bytes_per_iter = method_iteration_bytes(h, prec);
    h->stats.method_bytes_initial = method_initial_bytes(h, prec);
    if (herr) {
      HIPCHK(hipMemsetAsync(h->sync.err, 0, sizeof(unsigned), h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      return set_err(CPC_E_DEVICE, "a sweep wait exceeded its bound");
    }
    cpc_status status = CPC_OK;
    for (int s = 0; s < ns; ++s) {
      if (done[s] == DONE_BREAKDOWN) {
        status = set_err(CPC_E_BREAKDOWN, "PCG breakdown in system " + std::to_string(s));
        break;
      }
      if (done[s] != DONE_CONVERGED && done[s] != DONE_ZERO_RHS)
        status = set_err(CPC_E_MAXIT, "system " + std::to_string(s) + " did not converge within maxit");
    }
    h->stats.status = status;
    return status;
  } catch (const HipError& e) {
    return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
}

}  // namespace cpc

using namespace cpc;

namespace cpc {

cpc_status fail(cpc_status st, const char* msg) { return set_err(st, msg); }
int handle_device(const cpc_solver* h) { return h->device; }
bool handle_is_batch(const cpc_solver* h) { return h->batch; }

// The solve with the PCG scalars, the reduction partials and the sweep hand-off
// counters taken from caller-provided device memory instead of the handle's, and every
// iteration launched eagerly (no graph is instantiated, which would allocate). The
// handle's own pointers are swapped out for the duration of the call (a handle is used
// by one thread at a time) and put back on every exit path.
cpc_status run_solve_on_scratch(cpc_solver* h, const double* b, double* x, int use_x0, double tol, int maxit,
                                int32_t* iters, double* relres, const SolveScratch& sc) {
  struct Swap {
    cpc_solver* h;
    PcgState* st;
    double* partials;
    SweepSync sync;
    ~Swap() {
      h->st = st;
      h->partials = partials;
      h->sync = sync;
    }
  } keep{h, h->st, h->partials, h->sync};
  h->st = sc.st;
  h->partials = sc.partials;
  h->sync = sc.sync;
  // the memory keeps what the last call on this GPU left: the sweep counters must start
  // at zero (the PCG state is written whole before any kernel reads it, and every
  // reduction writes its partials before summing them)
  for (unsigned* c : {sc.sync.ticket, sc.sync.exited, sc.sync.err})
    if (hipMemsetAsync(c, 0, sizeof(unsigned), h->stream) != hipSuccess)
      return set_err(CPC_E_DEVICE, "clearing the sweep counters failed");
  return run_solve(h, h->opt.prec, b, x, use_x0, tol, maxit, iters, relres, true);
}

}  // namespace cpc

extern "C" {

void cpc_default_options(cpc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(cpc_options);
  o->prec = CPC_PREC_COMBINED;
  o->precision = CPC_FP64;
  o->max_coarse = 256;
  o->max_levels = 25;
  o->swap_roles = 0;
  o->check_symmetry = 1;
  o->use_graph = 1;
  o->check_every = 0;
  o->rap_on_gpu = 1;
  o->sweep_block_rows = 0;
  o->sweep_threads = 0;
  o->dense_smoother = 0;
  o->tune = 1;
  o->verbose = 0;
  o->ilu_fill = 0;
  o->theta = 0.25;
  o->sweep_kernel = 0;
}

const char* cpc_last_error(void) { return g_last_error.c_str(); }

static cpc_status read_options(const cpc_options* opt, cpc_options& o) {
  cpc_default_options(&o);
  if (opt) {
    if (opt->struct_size != (int32_t)sizeof(cpc_options)) return set_err(CPC_E_ARG, "cpc_options.struct_size mismatch");
    o = *opt;
  }
  if (o.prec < 0 || o.prec >= kNumPrec) return set_err(CPC_E_ARG, "unknown preconditioner");
  if (o.precision != CPC_FP64 && o.precision != CPC_FP32_PRECOND) return set_err(CPC_E_ARG, "unknown precision");
  if (o.max_levels < 1 || o.max_levels > 64 || o.max_coarse < 1) return set_err(CPC_E_ARG, "bad level limits");
  if (!(o.theta >= 0.0 && o.theta <= 1.0)) return set_err(CPC_E_ARG, "theta must lie in [0, 1]");
  if (o.sweep_threads != 0 && o.sweep_threads != 64 && o.sweep_threads != 256)
    return set_err(CPC_E_ARG, "sweep_threads must be 0, 64 or 256");
  if (o.dense_smoother < 0 || o.dense_smoother > 3) return set_err(CPC_E_ARG, "dense_smoother must be 0, 1, 2 or 3");
  if (o.ilu_fill < 0 || o.ilu_fill > 16) return set_err(CPC_E_ARG, "ilu_fill must lie in [0, 16]");
  if (o.sweep_kernel < 0 || o.sweep_kernel > 1) return set_err(CPC_E_ARG, "sweep_kernel must be 0 or 1");
  if (o.check_every < 0) return set_err(CPC_E_ARG, "check_every must be >= 0 (0: predicted)");
  return CPC_OK;
}

cpc_status cpc_setup(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                     const cpc_options* opt, void* hip_stream, cpc_handle* out) {
  if (!out) return set_err(CPC_E_ARG, "null output handle");
  *out = nullptr;
  cpc_options o;
  if (cpc_status os = read_options(opt, o)) return os;
  std::string msg;
  const double t0 = now_s();
  int vs = validate_csr(n, row_ptr, col_idx, val, o.check_symmetry != 0, &msg);
  if (vs != CPC_OK) return set_err((cpc_status)vs, msg);
  auto h = std::make_unique<cpc_solver>();
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;  // the setup's GPU calls report a missing device
  h->opt = o;
  h->setup_t0 = t0;
  h->n = n;
  h->nnz = row_ptr[n];
  h->f32 = (o.precision == CPC_FP32_PRECOND);
  try {
    // host-only work first: the input contract and ILU(0) are decided before any GPU call
    std::vector<SysHier> sys(1);
    {
      HostCsr A0;
      A0.n = n;
      A0.ncols = n;
      A0.rp.assign(row_ptr, row_ptr + n + 1);
      A0.ci.assign(col_idx, col_idx + row_ptr[n]);
      A0.v.assign(val, val + row_ptr[n]);
      sys[0].A.push_back(std::move(A0));
    }
    int st = ilu0_factor(sys[0].A[0], sys[0].lu, &msg);
    if (st != CPC_OK) return set_err((cpc_status)st, msg);
    if (o.ilu_fill > 0) {
      st = iluk_factor(sys[0].A[0], o.ilu_fill, h->iluF, h->iluF_lev, &msg);
      if (st != CPC_OK) return set_err((cpc_status)st, msg);
      h->iluk = true;
      for (int i = 0; i < n; ++i)
        for (int q = h->iluF.rp[i]; q < h->iluF.rp[i + 1]; ++q) (h->iluF.ci[q] < i ? h->ilu_lnnz : h->ilu_unnz) += 1.0;
    }
    if (hip_stream) {
      h->stream = (hipStream_t)hip_stream;
    } else {
      HIPCHK(hipStreamCreate(&h->stream));
      h->own_stream = true;
    }
    progress(h.get(), "ILU(0) factored; building the hierarchy");
    st = build_sys_hier(h.get(), sys[0], o, &msg);
    if (st != CPC_OK) return set_err((cpc_status)st, msg);
    progress(h.get(), "hierarchy of " + std::to_string(sys[0].A.size()) + " levels; assembling");
    st = assemble_levels(h.get(), sys, o, &msg);
    if (st != CPC_OK) return set_err((cpc_status)st, msg);
    sys.clear();
    allocate_work(h.get());
    progress(h.get(), "levels assembled; choosing smoother forms");
    tune_dense(h.get());
    tune_sweeps(h.get());
    if (h->iluk) {
      progress(h.get(), "ILU(" + std::to_string(o.ilu_fill) + ") sweeps");
      build_iluk_sweeps(h.get(), h->lev[0].sweep_R > 0 ? h->lev[0].sweep_R : choose_block_rows(n));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
  } catch (const HipError& e) {
    return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    return set_err(CPC_E_NOMEM, "host allocation failed");
  }
  h->stats.setup_s = now_s() - t0;
  *out = h.release();
  return CPC_OK;
}

cpc_status cpc_setup_batch(int32_t nsys, const int32_t* n, const int32_t* const* row_ptr,
                           const int32_t* const* col_idx, const double* const* val, const cpc_options* opt,
                           void* hip_stream, cpc_handle* out) {
  if (!out) return set_err(CPC_E_ARG, "null output handle");
  *out = nullptr;
  if (nsys < 1 || !n || !row_ptr || !col_idx || !val) return set_err(CPC_E_ARG, "bad batch arguments");
  cpc_options o;
  if (cpc_status os = read_options(opt, o)) return os;
  std::string msg;
  const double t0 = now_s();
  int64_t total = 0;
  for (int s = 0; s < nsys; ++s) {
    int vs = validate_csr(n[s], row_ptr[s], col_idx[s], val[s], o.check_symmetry != 0, &msg);
    if (vs != CPC_OK) return set_err((cpc_status)vs, "system " + std::to_string(s) + ": " + msg);
    total += n[s];
  }
  if (total > 2147483647LL) return set_err(CPC_E_ARG, "batch exceeds 2^31 rows");
  if (o.ilu_fill > 0) return set_err(CPC_E_ARG, "ilu_fill > 0 is offered for single systems only");
  auto h = std::make_unique<cpc_solver>();
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;  // the setup's GPU calls report a missing device
  h->opt = o;
  h->setup_t0 = t0;
  h->batch = true;
  h->nsys = nsys;
  h->f32 = (o.precision == CPC_FP32_PRECOND);
  try {
    std::vector<SysHier> sys(nsys);
    std::vector<int> sst(nsys, CPC_OK);
    std::vector<std::string> smsg(nsys);
    const int nthreads = setup_threads();
    progress(h.get(), "ILU(0) of " + std::to_string(nsys) + " systems on " + std::to_string(nthreads) +
                          " host threads");
    parallel_for(nsys, nthreads, [&](int s) {
      HostCsr A0;
      A0.n = A0.ncols = n[s];
      A0.rp.assign(row_ptr[s], row_ptr[s] + n[s] + 1);
      A0.ci.assign(col_idx[s], col_idx[s] + row_ptr[s][n[s]]);
      A0.v.assign(val[s], val[s] + row_ptr[s][n[s]]);
      sys[s].A.push_back(std::move(A0));
      sst[s] = ilu0_factor(sys[s].A[0], sys[s].lu, &smsg[s]);
    });
    for (int s = 0; s < nsys; ++s) {
      if (sst[s] != CPC_OK) return set_err((cpc_status)sst[s], "system " + std::to_string(s) + ": " + smsg[s]);
      h->sys_n.push_back(n[s]);
      h->sys_off.push_back(s == 0 ? 0 : h->sys_off[s - 1] + n[s - 1]);
    }
    h->n = (int)total;
    if (hip_stream) {
      h->stream = (hipStream_t)hip_stream;
    } else {
      HIPCHK(hipStreamCreate(&h->stream));
      h->own_stream = true;
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    // each system's hierarchy on a host thread: coarsening and interpolation on the host,
    // Galerkin products on a stream of the thread's own
    progress(h.get(), "hierarchies of " + std::to_string(nsys) + " systems on " + std::to_string(nthreads) +
                          " host threads");
    std::atomic<int> built{0};
    std::mutex plock;
    const int dev = h->device;
    parallel_for(nsys, nthreads, [&](int s) {
      hipStream_t ts = nullptr;
      try {
        HIPCHK(hipSetDevice(dev));
        HIPCHK(hipStreamCreate(&ts));
        sst[s] = build_sys_hier(h.get(), sys[s], o, &smsg[s], ts);
      } catch (const HipError& e) {
        sst[s] = CPC_E_DEVICE;
        smsg[s] = e.where + ": " + hipGetErrorString(e.e);
      }
      if (ts) (void)hipStreamDestroy(ts);
      const int k = ++built;
      if (k % 8 == 0 || k == nsys) {
        std::lock_guard<std::mutex> lock(plock);
        progress(h.get(), std::to_string(k) + " of " + std::to_string(nsys) + " hierarchies built");
      }
    });
    for (int s = 0; s < nsys; ++s)
      if (sst[s] != CPC_OK) return set_err((cpc_status)sst[s], "system " + std::to_string(s) + ": " + smsg[s]);
    progress(h.get(), "assembling the batch levels");
    int st = assemble_levels(h.get(), sys, o, &msg);
    if (st != CPC_OK) return set_err((cpc_status)st, msg);
    h->nnz = h->lev[0].A.nnz;
    sys.clear();
    allocate_work(h.get());
    allocate_batch(h.get());
    tune_dense(h.get());
    tune_sweeps(h.get());
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
  } catch (const HipError& e) {
    return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    return set_err(CPC_E_NOMEM, "host allocation failed");
  }
  h->stats.setup_s = now_s() - t0;
  *out = h.release();
  return CPC_OK;
}

cpc_status cpc_solve_batch(cpc_handle h, const double* b_dev, double* x_dev, double tol, int32_t maxit,
                           int32_t* iters, double* relres) {
  if (!h) return set_err(CPC_E_ARG, "null handle");
  return run_solve_batch(h, h->opt.prec, b_dev, x_dev, tol, maxit, iters, relres);
}

cpc_status cpc_batch_info(cpc_handle h, int32_t* nsys, int32_t* n, int32_t* offset) {
  if (!h) return set_err(CPC_E_ARG, "null handle");
  if (nsys) *nsys = h->nsys;
  for (int s = 0; s < h->nsys; ++s) {
    if (n) n[s] = h->batch ? h->sys_n[s] : h->n;
    if (offset) offset[s] = h->batch ? h->sys_off[s] : 0;
  }
  return CPC_OK;
}


cpc_status cpc_solve(cpc_handle h, const double* b_dev, double* x_dev, int32_t use_x0, double tol, int32_t maxit,
                     int32_t* iters, double* relres) {
  if (!h) return set_err(CPC_E_ARG, "null handle");
  if (h->batch) return set_err(CPC_E_ARG, "batch handle: use cpc_solve_batch");
  return run_solve(h, h->opt.prec, b_dev, x_dev, use_x0, tol, maxit, iters, relres);
}

cpc_status cpc_solve_with(cpc_handle h, int32_t prec, const double* b_dev, double* x_dev, int32_t use_x0, double tol,
                          int32_t maxit, int32_t* iters, double* relres) {
  return run_solve(h, prec, b_dev, x_dev, use_x0, tol, maxit, iters, relres);
}

cpc_status cpc_apply_op(cpc_handle h, int32_t op, const double* r_dev, double* z_dev) {
  if (!h) return set_err(CPC_E_ARG, "null handle");
  if (!r_dev || !z_dev) return set_err(CPC_E_ARG, "null vector");
  if (op < CPC_OP_COMBINED || op > CPC_OP_BBAR) return set_err(CPC_E_ARG, "unknown operator");
  try {
    apply_op(h, op, r_dev, z_dev, nullptr);
    HIPCHK(hipGetLastError());
    unsigned herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, h->sync.err, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (herr) {
      HIPCHK(hipMemsetAsync(h->sync.err, 0, sizeof(unsigned), h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      return set_err(CPC_E_DEVICE, "a sweep wait exceeded its bound");
    }
  } catch (const HipError& e) {
    return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
  return CPC_OK;
}

cpc_status cpc_spgemm(int32_t nrows, int32_t ninner, int32_t ncols, const int32_t* xrp, const int32_t* xci,
                      const double* xv, const int32_t* yrp, const int32_t* yci, const double* yv, int32_t* crp,
                      int32_t* cci, double* cv, int64_t* nnz) {
  if (nrows < 0 || ninner < 0 || ncols < 0 || !xrp || !yrp || !crp || !nnz)
    return set_err(CPC_E_ARG, "cpc_spgemm: bad sizes or null arrays");
  auto csr_ok = [](int n, int m, const int32_t* rp, const int32_t* ci, const double* v) {
    if (rp[0] != 0) return false;
    for (int i = 0; i < n; ++i)
      if (rp[i + 1] < rp[i]) return false;
    if (rp[n] > 0 && (!ci || !v)) return false;
    for (int q = 0; q < rp[n]; ++q)
      if (ci[q] < 0 || ci[q] >= m) return false;
    return true;
  };
  if (!csr_ok(nrows, ninner, xrp, xci, xv) || !csr_ok(ninner, ncols, yrp, yci, yv))
    return set_err(CPC_E_ARG, "cpc_spgemm: malformed CSR input");
  try {
    cpc_solver t;
    HIPCHK(hipStreamCreate(&t.stream));
    t.own_stream = true;
    HostCsr X, Y, C;
    X.n = nrows;
    X.ncols = ninner;
    X.rp.assign(xrp, xrp + nrows + 1);
    X.ci.assign(xci, xci + xrp[nrows]);
    X.v.assign(xv, xv + xrp[nrows]);
    Y.n = ninner;
    Y.ncols = ncols;
    Y.rp.assign(yrp, yrp + ninner + 1);
    Y.ci.assign(yci, yci + yrp[ninner]);
    Y.v.assign(yv, yv + yrp[ninner]);
    std::vector<void*> keep;
    DevCsr Xd, Yd, Cd;
    std::string msg;
    bool ok = false;
    try {
      upload_csr(&t, X, Xd, false, &keep, false);
      upload_csr(&t, Y, Yd, false, &keep, false);
      ok = gpu_spgemm(&t, Xd, Yd, ncols, C, Cd, &msg, keep);
      HIPCHK(hipStreamSynchronize(t.stream));
    } catch (...) {
      (void)hipStreamSynchronize(t.stream);
      for (void* p : keep) (void)hipFree(p);
      throw;
    }
    for (void* p : keep) (void)hipFree(p);
    if (!ok) return set_err(CPC_E_NOMEM, "cpc_spgemm: " + msg);
    std::copy(C.rp.begin(), C.rp.end(), crp);
    *nnz = C.rp[nrows];
    if (cci && cv) {
      std::copy(C.ci.begin(), C.ci.end(), cci);
      std::copy(C.v.begin(), C.v.end(), cv);
    }
  } catch (const HipError& e) {
    return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    return set_err(CPC_E_NOMEM, "host allocation failed");
  }
  return CPC_OK;
}

cpc_status cpc_spmv(cpc_handle h, int32_t level, const double* x_dev, double* y_dev) {
  if (!h) return set_err(CPC_E_ARG, "null handle");
  if (level < 0 || level >= (int)h->lev.size()) return set_err(CPC_E_ARG, "level out of range");
  if (!x_dev || !y_dev) return set_err(CPC_E_ARG, "null vector");
  try {
    const DevCsr& A = h->lev[level].A;
    spmv_or_throw(h, A.mat(false), 0, x_dev, false, nullptr, false, y_dev, false, A.tpr, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
  } catch (const HipError& e) {
    return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
  return CPC_OK;
}

cpc_status cpc_smoother_kind(cpc_handle h, int32_t level, int32_t* kind, int32_t* block_rows) {
  if (!h || !kind) return set_err(CPC_E_ARG, "null argument");
  if (level < 0 || level >= (int32_t)h->lev.size()) return set_err(CPC_E_ARG, "level out of range");
  const Level& L = h->lev[level];
  if (block_rows) *block_rows = L.sweep_R;
  if (L.nS <= 0 || level + 1 == (int32_t)h->lev.size()) *kind = -1;
  else *kind = L.dense_smooth ? 1 : (L.bdense ? 2 : 0);
  if (block_rows && L.bdense) *block_rows = L.bd.B;
  return CPC_OK;
}

cpc_status cpc_smoother_bytes(cpc_handle h, int32_t level, int64_t* bytes) {
  if (!h || !bytes) return set_err(CPC_E_ARG, "null argument");
  if (level < 0 || level >= (int32_t)h->lev.size()) return set_err(CPC_E_ARG, "level out of range");
  const Level& L = h->lev[level];
  double b = 0.0;
  if (L.nS > 0 && level + 1 < (int32_t)h->lev.size()) b = L.bdense ? L.bd.stored_bytes : (L.dense_smooth ? L.dense_bytes : 0.0);
  *bytes = (int64_t)b;
  return CPC_OK;
}

cpc_status cpc_hierarchy_info(cpc_handle h, int32_t* nlev, int32_t* n_l, int64_t* nnz_l, int32_t* depth_l) {
  if (!h) return set_err(CPC_E_ARG, "null handle");
  if (nlev) *nlev = (int32_t)h->lev.size();
  for (size_t d = 0; d < h->lev.size(); ++d) {
    if (n_l) n_l[d] = h->lev[d].A.n;
    if (nnz_l) nnz_l[d] = h->lev[d].A.nnz;
    if (depth_l) depth_l[d] = h->lev[d].lower.global_depth ? h->lev[d].lower.global_depth : lower_depth(h->lev[d].A_host);
  }
  return CPC_OK;
}

cpc_status cpc_get_level(cpc_handle h, int32_t level, int32_t* row_ptr, int32_t* col_idx, double* val) {
  if (!h) return set_err(CPC_E_ARG, "null handle");
  if (level < 0 || level >= (int)h->lev.size()) return set_err(CPC_E_ARG, "level out of range");
  const HostCsr& a = h->lev[level].A_host;
  if (row_ptr) std::memcpy(row_ptr, a.rp.data(), sizeof(int) * (a.n + 1));
  if (col_idx) std::memcpy(col_idx, a.ci.data(), sizeof(int) * a.nnz());
  if (val) std::memcpy(val, a.v.data(), sizeof(double) * a.nnz());
  return CPC_OK;
}

cpc_status cpc_get_prolongation(cpc_handle h, int32_t level, int64_t* p_nnz, int32_t* row_ptr, int32_t* col_idx,
                                double* val, int32_t* cf) {
  if (!h) return set_err(CPC_E_ARG, "null handle");
  if (level < 0 || level + 1 >= (int)h->lev.size()) return set_err(CPC_E_ARG, "level has no prolongation");
  const HostCsr& P = h->lev[level].P_host;
  if (p_nnz) *p_nnz = P.nnz();
  if (row_ptr) std::memcpy(row_ptr, P.rp.data(), sizeof(int) * (P.n + 1));
  if (col_idx) std::memcpy(col_idx, P.ci.data(), sizeof(int) * P.nnz());
  if (val) std::memcpy(val, P.v.data(), sizeof(double) * P.nnz());
  if (cf) std::memcpy(cf, h->lev[level].cf.data(), sizeof(int) * P.n);
  return CPC_OK;
}

cpc_status cpc_get_ilu(cpc_handle h, double* lu) {
  if (!h || !lu) return set_err(CPC_E_ARG, "null argument");
  if (h->iluk) return set_err(CPC_E_ARG, "the handle applies ILU(k), k > 0: use cpc_get_ilu_factor");
  std::memcpy(lu, h->lu_host.data(), sizeof(double) * h->lu_host.size());
  return CPC_OK;
}

cpc_status cpc_get_ilu_factor(cpc_handle h, int64_t* nnz, int32_t* row_ptr, int32_t* col_idx, double* val) {
  if (!h || !nnz) return set_err(CPC_E_ARG, "null argument");
  if (h->batch) return set_err(CPC_E_ARG, "batch handle");
  const HostCsr& A = h->lev[0].A_host;
  const std::vector<int>& rp = h->iluk ? h->iluF.rp : A.rp;
  const std::vector<int>& ci = h->iluk ? h->iluF.ci : A.ci;
  const std::vector<double>& v = h->iluk ? h->iluF.v : h->lu_host;
  *nnz = (int64_t)ci.size();
  if (row_ptr) std::memcpy(row_ptr, rp.data(), sizeof(int) * rp.size());
  if (col_idx) std::memcpy(col_idx, ci.data(), sizeof(int) * ci.size());
  if (val) std::memcpy(val, v.data(), sizeof(double) * v.size());
  return CPC_OK;
}

cpc_status cpc_get_stats(cpc_handle h, cpc_stats* st) {
  if (!h || !st) return set_err(CPC_E_ARG, "null argument");
  *st = h->stats;
  return CPC_OK;
}

cpc_status cpc_neg_outer_on_pattern(cpc_handle h, const double* lam_dev, const double* x_dev, double* g_nnz_dev) {
  if (!h || !lam_dev || !x_dev || !g_nnz_dev) return set_err(CPC_E_ARG, "null argument");
  try {
    launch_neg_outer(h->stream, h->lev[0].A.mat(false), lam_dev, x_dev, g_nnz_dev);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
  } catch (const HipError& e) {
    return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
  return CPC_OK;
}

cpc_status cpc_time_kernel(cpc_handle h, int32_t kernel, int32_t level, int32_t reps, double* avg_ms,
                           double* bytes_per_launch, int32_t* launches, double* form_bytes_per_launch) {
  if (!h) return set_err(CPC_E_ARG, "null handle");
  if (reps < 1 || kernel < CPC_K_SPMV_PQ || kernel > CPC_K_SWEEP) return set_err(CPC_E_ARG, "bad kernel or reps");
  const int nlev = (int)h->lev.size();
  const bool per_level = kernel >= CPC_K_FGS && kernel <= CPC_K_PROLONG && kernel != CPC_K_ILU_L &&
                         kernel != CPC_K_ILU_U;
  // levels the family runs on: smoothed levels (all but the coarsest), finest only for ILU/PCG
  std::vector<int> levels;
  // (kernel, level) launches of one repetition of the level-scheduled sweep family
  std::vector<std::pair<int, int>> mix;
  if (kernel == CPC_K_SWEEP) {
    // the triangular solves one B_co iteration runs as level-scheduled sweeps: per
    // smoothed level with sweeps the forward and backward sweep of each of the two
    // V-cycles, then the ILU(0) L and U solves
    for (int c = 0; c < 2; ++c)
      for (int d = 0; d + 1 < nlev; ++d)
        if (h->lev[d].nS > 0 && !h->lev[d].bdense && !h->lev[d].dense_smooth && (level < 0 || level == d)) {
          mix.push_back({CPC_K_FGS, d});
          mix.push_back({CPC_K_BGS, d});
        }
    if (level <= 0) {
      mix.push_back({CPC_K_ILU_L, 0});
      mix.push_back({CPC_K_ILU_U, 0});
    }
    if (mix.empty()) return set_err(CPC_E_ARG, "no level-scheduled sweep on that level");
  } else if (per_level) {
    if (level >= 0) {
      if (level >= nlev - 1 && !(nlev == 1 && level == 0 && kernel == CPC_K_RESIDUAL))
        return set_err(CPC_E_ARG, "level has no such kernel");
      levels.push_back(level);
    } else {
      for (int d = 0; d + 1 < nlev; ++d) levels.push_back(d);
    }
    if (levels.empty()) return set_err(CPC_E_ARG, "hierarchy has one level");
  } else if (kernel == CPC_K_DENSE_GEMV) {
    for (int d = 0; d + 1 < nlev; ++d)
      if ((h->lev[d].bdense || h->lev[d].dense_smooth) && (level < 0 || level == d)) levels.push_back(d);
    if (levels.empty()) return set_err(CPC_E_ARG, "no level is smoothed through explicit inverses");
  } else {
    levels.push_back(0);
  }
  const bool f32 = h->f32;
  const bool tri = kernel == CPC_K_FGS || kernel == CPC_K_BGS || kernel == CPC_K_ILU_L || kernel == CPC_K_ILU_U ||
                   kernel == CPC_K_SWEEP;
  // triangular solves are timed launch by launch (event pairs); the rest as one span
  std::vector<hipEvent_t> evs;
  bool timing = false;
  auto ev_begin = [&]() {
    if (!timing) return;
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    evs.push_back(e);
    HIPCHK(hipEventRecord(e, h->stream));
  };
  auto ev_end = ev_begin;
  // a pair of events for one launch that stamps them itself (null when not timing)
  auto ev_pair = [&](hipEvent_t& e0, hipEvent_t& e1) {
    e0 = e1 = nullptr;
    if (!timing) return;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    evs.push_back(e0);
    evs.push_back(e1);
  };
  auto launch_kernel = [&](int kern, int d) {
    Level& L = h->lev[d];
    void* f = d == 0 ? h->pin : L.f;
    void* u = d == 0 ? h->u1 : L.u;
    switch (kern) {
      case CPC_K_SPMV_PQ:
        launch_spmv_pq(h->stream, L.A.mat(false), h->p, h->q, h->partials, h->st, L.A.tpr);
        break;
      // triangular solves: the sentinel fill before each launch is not timed
      case CPC_K_FGS:
        if (L.bdense) {
          ev_begin();
          bdense_solve(h, L, false, f, u, L.r, nullptr);
          ev_end();
          break;
        }
        if (L.dense_smooth) {
          ev_begin();
          launch_dense_lower(h->stream, L.dtri, f32, f32, f, u, nullptr);
          ev_end();
          break;
        }
        launch_fill_sentinel(h->stream, L.lower.d.n, u, f32, nullptr);
        {
          hipEvent_t e0, e1;
          ev_pair(e0, e1);
          launch_tri(h, SWEEP_LOWER, L.lower, L.fgs, f, u, nullptr, nullptr, nullptr, e0, e1);
        }
        break;
      case CPC_K_BGS:
        if (L.bdense) {
          ev_begin();
          bdense_solve(h, L, true, f, u, L.r, nullptr);
          ev_end();
          break;
        }
        if (L.dense_smooth) {
          ev_begin();
          launch_dense_lower_t(h->stream, L.dtri, f32, f32, f, u, nullptr);
          ev_end();
          break;
        }
        launch_fill_sentinel(h->stream, L.upper.d.n, u, f32, nullptr);
        {
          hipEvent_t e0, e1;
          ev_pair(e0, e1);
          launch_tri(h, SWEEP_UPPER, L.upper, L.bgs, f, u, nullptr, nullptr, nullptr, e0, e1);
        }
        break;
      case CPC_K_ILU_L:
        launch_fill_sentinel(h->stream, ilu_lower_sched(h).d.n, h->y, f32, nullptr);
        {
          hipEvent_t e0, e1;
          ev_pair(e0, e1);
          launch_tri(h, SWEEP_UNIT_LOWER, ilu_lower_sched(h), h->ilu_l, h->res, h->y, nullptr, nullptr, nullptr, e0,
                     e1);
        }
        break;
      case CPC_K_ILU_U:
        launch_fill_sentinel(h->stream, ilu_upper_sched(h).d.n, h->w, f32, nullptr);
        {
          hipEvent_t e0, e1;
          ev_pair(e0, e1);
          launch_tri(h, SWEEP_UPPER_OUT, ilu_upper_sched(h), h->ilu_u, h->y, h->w, h->u1, h->u2, nullptr, e0, e1);
        }
        break;
      case CPC_K_RESIDUAL:
        spmv_or_throw(h, smoothed(L.A, L.nS, f32), 1, u, f32, f, f32, L.r, f32, L.A.tpr, nullptr);
        break;
      case CPC_K_RESTRICT:
        spmv_or_throw(h, L.R.mat(f32), 0, L.r, f32, nullptr, f32, h->lev[d + 1].f, f32, L.R.tpr, nullptr);
        break;
      case CPC_K_PROLONG:
        spmv_or_throw(h, L.P.mat(f32), 2, h->lev[d + 1].u, f32, nullptr, f32, u, f32, L.P.tpr, nullptr);
        break;
      case CPC_K_VCYCLE:
        vcycle(h, 0, h->pin, h->u1, nullptr);
        break;
      case CPC_K_PRECOND:
        apply_op(h, prec_to_op(h->opt.prec), h->r, h->z, nullptr);
        break;
      default:
        enqueue_iteration(h, h->opt.prec, h->z64tmp);
        break;
    }
  };
  auto launch_once = [&](int d) {
    if (kernel == CPC_K_SWEEP) {
      for (const auto& km : mix) launch_kernel(km.first, km.second);
    } else {
      launch_kernel(kernel, d);
    }
  };
  if (kernel == CPC_K_DENSE_GEMV) {
    // the dense products of every selected level, both directions (one launch per
    // block and direction), each launch stamping its own start and end into a pair of
    // events, so that the mean is that of the kernels, not of the gaps between them
    std::vector<hipEvent_t> pool;
    try {
      double bytes = 0.0, mbytes = 0.0;
      const double eb = f32 ? 4.0 : 8.0, vb = f32 ? 4.0 : 8.0;
      // the method's share: the forward and backward triangular solves these products
      // evaluate, spread over their launches
      for (int d : levels) mbytes += method_kernel_bytes(h, CPC_K_FGS, d) + method_kernel_bytes(h, CPC_K_BGS, d);
      struct Item {
        int level, dir, step;  // step of the block-dense form, or -1 for a whole-level inverse
      };
      std::vector<Item> items;
      for (int d : levels) {
        const Level& L = h->lev[d];
        for (int dir = 0; dir < 2; ++dir) {
          const int T = L.bdense ? bd_steps(L, dir == 1) : 1;
          for (int t = 0; t < T; ++t) {
            items.push_back({d, dir, L.bdense ? t : -1});
            if (!L.bdense) {
              bytes += eb * L.dense_entries + 2.0 * vb * L.nS;
              continue;
            }
            const std::vector<int>& step = dir == 1 ? L.bd.bstep : L.bd.fstep;
            for (int q = step[t]; q < step[t + 1]; ++q) {
              const double nb = L.bd.rows[dir == 1 ? L.bd.bblk[q] : q];
              bytes += eb * 0.5 * nb * (nb + 1) + 2.0 * vb * nb;
            }
          }
        }
      }
      const int count = (int)items.size();
      pool.resize(2 * (size_t)count);
      for (auto& e : pool) HIPCHK(hipEventCreate(&e));
      auto pass = [&](bool timed) {
        int q = 0;
        for (const auto& it : items) {
          Level& L = h->lev[it.level];
          void* f = it.level == 0 ? h->pin : L.f;
          void* u = it.level == 0 ? h->u1 : L.u;
          const DenseTriDev dt = it.step >= 0 ? bd_step(L, it.dir == 1, it.step) : L.dtri;
          hipEvent_t e0 = timed ? pool[2 * q] : nullptr, e1 = timed ? pool[2 * q + 1] : nullptr;
          ++q;
          if (it.dir == 0) launch_dense_lower(h->stream, dt, f32, f32, f, u, nullptr, e0, e1);
          else launch_dense_lower_t(h->stream, dt, f32, f32, f, u, nullptr, e0, e1);
        }
      };
      pass(false);  // warm-up
      double ms = 0.0;
      for (int r = 0; r < reps; ++r) {
        pass(true);
        HIPCHK(hipEventSynchronize(pool.back()));
        for (int q = 0; q < count; ++q) {
          float t = 0.f;
          HIPCHK(hipEventElapsedTime(&t, pool[2 * q], pool[2 * q + 1]));
          ms += t;
        }
      }
      for (auto& e : pool) (void)hipEventDestroy(e);
      pool.clear();
      if (avg_ms) *avg_ms = ms / ((double)reps * count);
      if (bytes_per_launch) *bytes_per_launch = mbytes / count;
      if (form_bytes_per_launch) *form_bytes_per_launch = bytes / count;
      if (launches) *launches = reps * count;
      HIPCHK(hipGetLastError());
    } catch (const HipError& e) {
      for (auto& ev : pool) (void)hipEventDestroy(ev);
      return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
    }
    return CPC_OK;
  }
  try {
    if (kernel == CPC_K_SWEEP) levels.assign(1, 0);  // one repetition = the whole mix
    if (kernel == CPC_K_SPMV_PQ || kernel == CPC_K_ITERATION) {
      // a running state with positive scalars so that nothing returns early
      PcgState s{};
      s.rz = 1.0;
      s.bb = 1.0;
      s.tol = 0.0;
      s.maxit = 1 << 30;
      HIPCHK(hipMemcpyAsync(h->st, &s, sizeof(s), hipMemcpyHostToDevice, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    for (int d : levels) launch_once(d);  // warm-up
    timing = true;
    if (!tri) ev_begin();
    for (int r = 0; r < reps; ++r)
      for (int d : levels) launch_once(d);
    if (!tri) ev_end();
    HIPCHK(hipEventSynchronize(evs.back()));
    float ms = 0.f;
    for (size_t k = 0; k + 1 < evs.size(); k += 2) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, evs[k], evs[k + 1]));
      ms += t;
    }
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    evs.clear();
    HIPCHK(hipGetLastError());
    double b = 0.0, fb = 0.0;
    int per_rep = (int)levels.size();
    if (kernel == CPC_K_SWEEP) {
      for (const auto& km : mix) {
        b += method_kernel_bytes(h, km.first, km.second);
        fb += kernel_bytes(h, km.first, km.second);
      }
      per_rep = (int)mix.size();
    } else {
      for (int d : levels) {
        if (kernel <= CPC_K_PROLONG) {
          b += method_kernel_bytes(h, kernel, d);
          fb += kernel_bytes(h, kernel, d);
        } else if (kernel == CPC_K_VCYCLE) {
          b += method_vcycle_bytes(h);
          fb += vcycle_bytes(h);
        } else if (kernel == CPC_K_PRECOND) {
          b += method_prec_bytes(h, h->opt.prec);
          fb += prec_bytes(h, h->opt.prec);
        } else {
          b += method_iteration_bytes(h, h->opt.prec);
          fb += iteration_bytes(h, h->opt.prec);
        }
      }
    }
    const int nl = reps * per_rep;
    if (avg_ms) *avg_ms = ms / nl;
    if (bytes_per_launch) *bytes_per_launch = b / per_rep;
    if (form_bytes_per_launch) *form_bytes_per_launch = fb / per_rep;
    if (launches) *launches = nl;
    unsigned herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, h->sync.err, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (herr) {
      HIPCHK(hipMemsetAsync(h->sync.err, 0, sizeof(unsigned), h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      return set_err(CPC_E_DEVICE, "a sweep wait exceeded its bound");
    }
  } catch (const HipError& e) {
    return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
  return CPC_OK;
}

cpc_status cpc_set_operator_values(cpc_handle h, const double* val_dev) {
  if (!h) return set_err(CPC_E_ARG, "null handle");
  if (h->op_vals != val_dev) {
    h->op_vals = val_dev;
    for (int i = 0; i < kNumPrec; ++i) {  // captured graphs bind the operator's values
      if (h->graph[i]) (void)hipGraphExecDestroy(h->graph[i]);
      if (h->graph_src[i]) (void)hipGraphDestroy(h->graph_src[i]);
      h->graph[i] = nullptr;
      h->graph_src[i] = nullptr;
      h->graph_x[i] = nullptr;
    }
  }
  return CPC_OK;
}

cpc_status cpc_tpfa_pattern(int32_t nx, int32_t ny, int32_t nz, int32_t* row_ptr, int32_t* col_idx) {
  if (nx < 1 || ny < 1 || nz < 1 || !row_ptr) return set_err(CPC_E_ARG, "bad grid or null row_ptr");
  const int64_t N = (int64_t)nx * ny * nz;
  if (N * 7 > 2147483647LL) return set_err(CPC_E_ARG, "grid too large for int32 indices");
  const int64_t nxy = (int64_t)nx * ny;
  int64_t p = 0;
  row_ptr[0] = 0;
  for (int64_t c = 0; c < N; ++c) {
    const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / nxy);
    const int64_t nb[7] = {k > 0 ? c - nxy : -1, j > 0 ? c - nx : -1, i > 0 ? c - 1 : -1, c,
                           i < nx - 1 ? c + 1 : -1, j < ny - 1 ? c + nx : -1, k < nz - 1 ? c + nxy : -1};
    for (int t = 0; t < 7; ++t)
      if (nb[t] >= 0) {
        if (col_idx) col_idx[p] = (int32_t)nb[t];
        ++p;
      }
    row_ptr[c + 1] = (int32_t)p;
  }
  return CPC_OK;
}

cpc_status cpc_tpfa_values(int32_t nx, int32_t ny, int32_t nz, double kz_ratio, int32_t dirichlet_x,
                           const double* logk_dev, const int32_t* row_ptr_dev, double* val_dev, void* hip_stream) {
  if (nx < 1 || ny < 1 || nz < 1 || !logk_dev || !row_ptr_dev || !val_dev || !(kz_ratio > 0.0))
    return set_err(CPC_E_ARG, "bad grid, null pointer or kz_ratio <= 0");
  try {
    launch_tpfa_values((hipStream_t)hip_stream, nx, ny, nz, kz_ratio, dirichlet_x, logk_dev, row_ptr_dev, val_dev);
    HIPCHK(hipGetLastError());
  } catch (const HipError& e) {
    return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
  return CPC_OK;
}

cpc_status cpc_tpfa_logk_grad(int32_t nx, int32_t ny, int32_t nz, double kz_ratio, int32_t dirichlet_x,
                              const double* logk_dev, const double* lam_dev, const double* x_dev, double* grad_dev,
                              void* hip_stream) {
  if (nx < 1 || ny < 1 || nz < 1 || !logk_dev || !lam_dev || !x_dev || !grad_dev || !(kz_ratio > 0.0))
    return set_err(CPC_E_ARG, "bad grid, null pointer or kz_ratio <= 0");
  try {
    launch_tpfa_grad((hipStream_t)hip_stream, nx, ny, nz, kz_ratio, dirichlet_x, logk_dev, lam_dev, x_dev, grad_dev);
    HIPCHK(hipGetLastError());
  } catch (const HipError& e) {
    return set_err(CPC_E_DEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
  return CPC_OK;
}

void cpc_destroy(cpc_handle h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

}  // extern "C"
