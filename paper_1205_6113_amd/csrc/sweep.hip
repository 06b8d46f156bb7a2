// Persistent, block-pipelined, level-scheduled triangular solve over packed rows:
// forward (D+L) and (I+L) solves, backward (D+U) solves, the building blocks of the
// Gauss-Seidel smoother and of ILU(0) application.
//
// Rows are cut into contiguous blocks; a workgroup takes blocks from a ticket counter
// in dependency order and walks the block's levels (sets of rows whose dependencies
// all lie in earlier levels or in blocks taken earlier). The block's row list, entry
// offsets and per-level ranges are staged in LDS, and the block's solved values are
// kept in LDS for the block's own later levels.
//
// One level takes two phases. Phase A: the level's dependency entries are contiguous
// in the pack, so the NT lanes split them evenly, each multiplying its entries by the
// solved values and writing the products to LDS. Phase B: groups of TB lanes add up
// one row's products in a fixed order, and the group's first lane scales by the
// reciprocal diagonal and stores the value in LDS and in the global vector. With one
// wave per workgroup (NT = 64, used where one block covers the matrix) the barriers
// between the phases reduce to LDS waits.
//
// Entry data are prefetched four levels ahead into a ring of register slots, with
// addresses taken from LDS (the vector-memory counter completes in order, so a load
// whose address comes from another load in flight would drain every younger
// prefetch); the LDS reads of a prefetch overlap the phases of the current level.
// Values from other blocks are first read two levels ahead. The output vector starts
// filled with a sentinel bit pattern, so a value that is not the sentinel is final; a
// read that still finds the sentinel polls the same address until the other block has
// stored the value (bounded: past the spin limit the error flag is set). No progress
// counters, cache-wide fences or extra hand-off loads are needed.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "wave_sum.hpp"

namespace cpc {

namespace {

constexpr int kNT = 256;  // threads of the fill kernel and of a multi-wave sweep workgroup
constexpr int kBudget = 150 * 1024;
// prefetched entries per lane and level: 1024 per level for 4 waves, 512 for one
constexpr int kp_of(int nt) { return nt == 64 ? 8 : 4; }

__device__ __forceinline__ bool is_sentinel(double v) {
  return (unsigned long long)__double_as_longlong(v) == kSentinel64;
}
__device__ __forceinline__ bool is_sentinel(float v) { return __float_as_uint(v) == kSentinel32; }

// Makes the compiler complete the loads of v here, where the number of loads issued
// since is known, rather than at a later use that follows loops with loads of their own
// (after which the wait it can prove safe is a full drain of every prefetch).
template <typename T>
__device__ __forceinline__ void settle(const T& v) {
  asm volatile("" ::"v"(v));
}

template <typename VT, typename XT, int KP>
struct Slot {
  int E0, E1, q0, q1;  // level's entry range and row range (block-relative positions)
  int col[KP];
  VT val[KP];
  XT xr[KP];      // values from other blocks (possibly still the sentinel)
  int row, a, n;  // the first-pass row of this lane's group, its products' offset and count
  XT fv, bv;
  VT dinv;        // reciprocal diagonal
};

template <int OP, int TB, int NT, typename VT, typename XT>
__global__ __launch_bounds__(NT) void tri_sweep_kernel(SweepDev sw, SweepPackDev pk, const XT* __restrict__ f,
                                                       XT* x, const XT* __restrict__ base, XT* __restrict__ out,
                                                       SweepSync sy, const int* __restrict__ done, long spin_limit) {
  constexpr bool FWD = (OP == SWEEP_LOWER || OP == SWEEP_UNIT_LOWER);
  constexpr bool UNIT = (OP == SWEEP_UNIT_LOWER);
  constexpr bool OUT = (OP == SWEEP_UPPER_OUT);
  constexpr int KP = kp_of(NT);
  constexpr int NG = NT / TB;
  using S = Slot<VT, XT, KP>;
  extern __shared__ unsigned char smem_raw[];
  double* prod = reinterpret_cast<double*>(smem_raw);
  XT* xs = reinterpret_cast<XT*>(smem_raw + sw.off_xs);
  int* rows_l = reinterpret_cast<int*>(smem_raw + sw.off_rows);
  int* ptr_l = reinterpret_cast<int*>(smem_raw + sw.off_ptr);
  int4* meta = reinterpret_cast<int4*>(smem_raw + sw.off_meta);
  __shared__ int s_tick;
  __shared__ int s_last;
  if (done && *done) return;  // before taking a ticket: the counters stay untouched
  const int tid = threadIdx.x;
  const int g = tid / TB, lane = tid % TB;
  const VT* __restrict__ pval = reinterpret_cast<const VT*>(pk.val);
  const VT* __restrict__ pdinv = reinterpret_cast<const VT*>(pk.diag);

  for (;;) {
    if (tid == 0) s_tick = (int)atomicAdd(sy.ticket, 1u);
    __syncthreads();
    const int t = s_tick;
    __syncthreads();
    if (t >= sw.nblk) break;
    const int b = FWD ? t : sw.nblk - 1 - t;
    if (masked(sw.mask, b)) continue;  // a block of a system that has stopped
    const int r0 = sw.blk_row[b], r1 = sw.blk_row[b + 1];
    const int nb = r1 - r0;
    const int lb = sw.blk_beg[b];
    const int nl = sw.blk_end[b] - lb;
    const int P0 = sw.lvl_ptr[lb];
    for (int q = tid; q < nb; q += NT) rows_l[q] = pk.row[P0 + q];
    for (int q = tid; q <= nb; q += NT) ptr_l[q] = pk.ptr[P0 + q];
    __syncthreads();
    // per level: rows [q0, q1) and dependency entries [E0, E1)
    for (int m = tid; m < nl; m += NT) {
      const int q0 = sw.lvl_ptr[lb + m] - P0, q1 = sw.lvl_ptr[lb + m + 1] - P0;
      meta[m] = make_int4(q0, q1, ptr_l[q0], ptr_l[q1]);
    }
    __syncthreads();

    // LDS part of the prefetch of level m: the level's ranges and, for this lane's group,
    // its first-pass row and that row's entry range
    struct Pre {
      int4 mt;
      bool has;              // the group has a first-pass row
      int qc, row, p0, p1;   // its position (or a valid dummy), row and entry range
    };
    auto pre_meta = [&](int m) -> int4 { return m < nl ? meta[m] : make_int4(0, 0, 0, 0); };
    auto pre_rows = [&](const int4& mt) -> Pre {
      Pre p;
      p.mt = mt;
      const int q = mt.x + g;
      p.has = q < mt.y;
      p.qc = p.has ? q : 0;
      p.row = rows_l[p.qc];
      p.p0 = ptr_l[p.qc];
      p.p1 = ptr_l[p.qc + 1];
      return p;
    };
    // global part: entries of the level and the first-pass row's data (dummy but valid
    // addresses where there is nothing to load, so that every step issues the same loads)
    auto issue = [&](S& s, const Pre& p) {
      const int E0 = p.mt.z, E1 = p.mt.w;
      s.E0 = E0;
      s.E1 = E1;
      s.q0 = p.mt.x;
      s.q1 = p.mt.y;
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const int e = E0 + tid + k * NT;
        const int ec = e < E1 ? e : 0;
        s.col[k] = pk.col[ec];
        s.val[k] = pval[ec];
      }
      s.row = p.has ? p.row : -1;
      s.a = p.p0 - E0;
      s.n = p.p1 - p.p0;
      s.fv = f[p.row];
      if (!UNIT) s.dinv = pdinv[P0 + p.qc];
      if (OUT) s.bv = base[p.row];
    };
    // first reads of the values a level takes from other blocks: plain loads, issued
    // only for such entries. The output was filled with the sentinel by an earlier
    // kernel, so a plain load returns the sentinel or the final value; only the polls
    // that follow a sentinel need agent-scope loads.
    auto issue_remote = [&](S& s) {
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const int e = s.E0 + tid + k * NT;
        const int c = s.col[k];
        if (e < s.E1 && c < 0) s.xr[k] = x[-(c + 1)];
      }
    };
    // poll until another block has stored x[j]; every exit follows a test of the last
    // value loaded, so no load is left in flight past the loop
    auto ready = [&](XT v, int j) -> double {
      long spins = 0;
      while (is_sentinel(v)) {
        if (++spins > spin_limit) {
          atomicOr(sy.err, 1u);
          break;
        }
        if ((spins & 255) == 0 && __hip_atomic_load(sy.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(x + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      return (double)v;
    };
    auto finish = [&](int i, double sum, double fv, double dinv, double bv) {
      const double xi = UNIT ? fv - sum : (fv - sum) * dinv;
      const XT xo = (XT)xi;
      xs[i - r0] = xo;
      __hip_atomic_store(x + i, xo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (OUT) out[i] = (XT)(bv + (double)xo);
    };
    // phase A: products of the level's entries into LDS (or, for a level of one row
    // longer than the product slots, per-lane partial sums)
    auto phase_a = [&](const S& s) -> bool {
      const int E0 = s.E0, E1 = s.E1;
      const bool lng = (E1 - E0) > sw.pcap;
      double part = 0.0;
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const int e = E0 + tid + k * NT;
        if (e < E1) {
          const int c = s.col[k];
          const double xv = c >= 0 ? (double)xs[c] : ready(s.xr[k], -(c + 1));
          const double pr = (double)s.val[k] * xv;
          if (lng) part += pr;
          else prod[e - E0] = pr;
        }
      }
      for (int e = E0 + tid + KP * NT; e < E1; e += NT) {
        const int c = pk.col[e];
        double xv;
        if (c >= 0) xv = (double)xs[c];
        else xv = ready(__hip_atomic_load(x + (-(c + 1)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), -(c + 1));
        const double pr = (double)pval[e] * xv;
        if (lng) part += pr;
        else prod[e - E0] = pr;
      }
      if (lng) prod[tid] = part;
      return lng;
    };
    // phase B: row sums in a fixed order, then the solved values
    auto phase_b = [&](const S& s, bool lng) {
      const double fv = (double)s.fv, dinv = UNIT ? 1.0 : (double)s.dinv, bv = OUT ? (double)s.bv : 0.0;
      if (lng) {
        if (g == 0) {
          double acc = 0.0;
          for (int j = lane; j < NT; j += TB) acc += prod[j];
          acc = gsum<TB>(acc);
          if (lane == 0) finish(s.row, acc, fv, dinv, bv);
        }
        return;
      }
      if (s.row >= 0) {  // first pass: the rows whose data were prefetched
        double acc = 0.0;
        for (int j = lane; j < s.n; j += TB) acc += prod[s.a + j];
        acc = gsum<TB>(acc);
        if (lane == 0) finish(s.row, acc, fv, dinv, bv);
      }
      for (int q2 = s.q0 + g + NG; q2 < s.q1; q2 += NG) {  // levels with more rows than groups
        const int a = ptr_l[q2] - s.E0, len = ptr_l[q2 + 1] - ptr_l[q2];
        double acc = 0.0;
        for (int j = lane; j < len; j += TB) acc += prod[a + j];
        acc = gsum<TB>(acc);
        if (lane == 0) {
          const int i = rows_l[q2];
          finish(i, acc, (double)f[i], UNIT ? 1.0 : (double)pdinv[P0 + q2], OUT ? (double)base[i] : 0.0);
        }
      }
    };
    // one level m (slot s); the LDS reads of level m + 4's prefetch overlap the level's
    // phases, its loads follow, and the other-block values of level m + 2 (slot s2)
    auto step = [&](S& s, S& s2, int m) {
      const int4 mt = pre_meta(m + 4);
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        settle(s.col[k]);
        settle(s.val[k]);
        settle(s.xr[k]);
        settle(s2.col[k]);
      }
      settle(s.fv);
      if (!UNIT) settle(s.dinv);
      if (OUT) settle(s.bv);
      const bool lng = phase_a(s);
      __syncthreads();
      const Pre p = pre_rows(mt);
      phase_b(s, lng);
      __syncthreads();
      issue_remote(s2);
      issue(s, p);
    };

    S s0, s1, s2, s3;
    issue(s0, pre_rows(pre_meta(0)));
    issue(s1, pre_rows(pre_meta(1)));
    issue(s2, pre_rows(pre_meta(2)));
    issue(s3, pre_rows(pre_meta(3)));
    issue_remote(s0);
    issue_remote(s1);
    for (int m = 0; m < nl; m += 4) {  // every step runs (levels past nl are empty) so that
      step(s0, s2, m);                 // each iteration issues the same loads
      step(s1, s3, m + 1);
      step(s2, s0, m + 2);
      step(s3, s1, m + 3);
    }
  }
  if (tid == 0) s_last = (atomicAdd(sy.exited, 1u) == gridDim.x - 1);
  __syncthreads();
  if (s_last && tid == 0) {
    *sy.ticket = 0u;
    *sy.exited = 0u;
  }
}

template <typename XT>
__global__ __launch_bounds__(kNT) void fill_sentinel_kernel(int n, XT* __restrict__ x, const int* __restrict__ done) {
  if (done && *done) return;
  for (int i = blockIdx.x * kNT + threadIdx.x; i < n; i += gridDim.x * kNT) {
    if constexpr (sizeof(XT) == 8) reinterpret_cast<unsigned long long*>(x)[i] = kSentinel64;
    else reinterpret_cast<unsigned*>(x)[i] = kSentinel32;
  }
}

template <int OP, int TB, int NT, typename VT, typename XT>
void launch_one(hipStream_t s, const SweepDev& sw, const SweepPackDev& pk, const void* f, void* x,
                const void* base, void* out, const SweepSync& sync, const int* done, long spin_limit) {
  static int attr = 65536;  // dynamic LDS the kernel may use without an attribute
  if (sw.lds > attr) {
    if (hipFuncSetAttribute((const void*)tri_sweep_kernel<OP, TB, NT, VT, XT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kBudget) != hipSuccess) {
      (void)hipGetLastError();  // leave no sticky error; the launch below reports the failure
    } else {
      attr = kBudget;
    }
  }
  tri_sweep_kernel<OP, TB, NT, VT, XT><<<sw.grid, NT, sw.lds, s>>>(sw, pk, (const XT*)f, (XT*)x, (const XT*)base,
                                                                   (XT*)out, sync, done, spin_limit);
}

template <int OP, int NT, typename VT, typename XT>
void dispatch_tb(hipStream_t s, const SweepDev& sw, const SweepPackDev& pk, const void* f, void* x,
                 const void* base, void* out, const SweepSync& sync, const int* done, long spin_limit) {
  switch (pk.tb) {
    case 1: launch_one<OP, 1, NT, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    case 2: launch_one<OP, 2, NT, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    case 4: launch_one<OP, 4, NT, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    case 8: launch_one<OP, 8, NT, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    case 16: launch_one<OP, 16, NT, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    case 32: launch_one<OP, 32, NT, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    default: launch_one<OP, 64, NT, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
  }
}

template <int OP, typename VT, typename XT>
void dispatch_nt(hipStream_t s, const SweepDev& sw, const SweepPackDev& pk, const void* f, void* x,
                 const void* base, void* out, const SweepSync& sync, const int* done, long spin_limit) {
  if (sw.nt == 64) dispatch_tb<OP, 64, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit);
  else dispatch_tb<OP, kNT, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit);
}

}  // namespace

int sweep_max_rows_per_block() { return 8192; }
int sweep_lds_budget() { return kBudget; }
int sweep_threads() { return kNT; }

void launch_sweep_packed(hipStream_t s, int op, const SweepDev& sw, const SweepPackDev& pk, bool fp32,
                         const void* f, void* x, const void* base, void* out, const SweepSync& sync,
                         const int* done, long spin_limit) {
  if (sw.n <= 0) return;
#define CPC_SW(OPC)                                                                                    \
  if (fp32) dispatch_nt<OPC, float, float>(s, sw, pk, f, x, base, out, sync, done, spin_limit);     \
  else dispatch_nt<OPC, double, double>(s, sw, pk, f, x, base, out, sync, done, spin_limit);
  switch (op) {
    case SWEEP_LOWER: CPC_SW(SWEEP_LOWER) break;
    case SWEEP_UPPER: CPC_SW(SWEEP_UPPER) break;
    case SWEEP_UNIT_LOWER: CPC_SW(SWEEP_UNIT_LOWER) break;
    default: CPC_SW(SWEEP_UPPER_OUT) break;
  }
#undef CPC_SW
}

void launch_fill_sentinel(hipStream_t s, int n, void* x, bool fp32, const int* done) {
  if (n <= 0) return;
  const int grid = std::min((n + kNT - 1) / kNT, 2048);
  if (fp32) fill_sentinel_kernel<float><<<grid, kNT, 0, s>>>(n, (float*)x, done);
  else fill_sentinel_kernel<double><<<grid, kNT, 0, s>>>(n, (double*)x, done);
}

}  // namespace cpc
