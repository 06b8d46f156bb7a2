// Persistent, block-pipelined, level-scheduled triangular solve over packed rows:
// forward (D+L) and (I+L) solves, backward (D+U) solves, the building blocks of the
// Gauss-Seidel smoother and of ILU(0) application.
//
// Rows are cut into contiguous blocks; a workgroup takes blocks from a ticket counter
// in dependency order and walks the block's levels (sets of rows whose dependencies
// all lie in earlier levels or in blocks taken earlier). The block's level table, row
// list and entry offsets are staged in LDS, and the block's solved values are kept in
// LDS for the block's own later levels.
//
// One level takes two phases. Phase A: the level's dependency entries are contiguous
// in the pack, so the 256 lanes split them evenly, each multiplying its entries by the
// solved values and writing the products to LDS. Phase B: groups of TB lanes add up
// one row's products in a fixed order, and the group's first lane divides by the
// diagonal and stores the value in LDS and in the global vector.
//
// Entry data are prefetched four levels ahead into a ring of register slots, with
// addresses taken from LDS (the vector-memory counter completes in order, so a load
// whose address comes from another load in flight would drain every younger
// prefetch). Values from other blocks are read with agent-scope loads issued two
// levels ahead. The output vector starts filled with a sentinel bit pattern, so a
// value that is not the sentinel is final; a read that still finds the sentinel polls
// the same address until the other block has stored the value (bounded: past the
// spin limit the error flag is set). No progress counters, cache-wide fences or
// extra hand-off loads are needed.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace cpc {

namespace {

constexpr int kNT = 256;  // threads per workgroup
constexpr int kKP = 4;    // prefetched entries per lane and level
constexpr int kBudget = 150 * 1024;

__device__ __forceinline__ bool is_sentinel(double v) {
  return (unsigned long long)__double_as_longlong(v) == kSentinel64;
}
__device__ __forceinline__ bool is_sentinel(float v) { return __float_as_uint(v) == kSentinel32; }

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of W lanes; the total is valid in each group's first lane.
// Lane exchanges: xor 1, xor 2 (quad permutations), mirror within 8 and within 16
// (DPP), xor 16 within 32 (swizzle), lane 32 read into lane 0.
template <int W>
__device__ __forceinline__ double gsum(double v) {
  if constexpr (W >= 2) v += dpp<0xB1>(v);
  if constexpr (W >= 4) v += dpp<0x4E>(v);
  if constexpr (W >= 8) v += dpp<0x141>(v);
  if constexpr (W >= 16) v += dpp<0x140>(v);
  if constexpr (W >= 32) {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
    v += __hiloint2double(hi, lo);
  }
  if constexpr (W >= 64)
    v += __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 32),
                          __builtin_amdgcn_readlane(__double2loint(v), 32));
  return v;
}

template <typename VT, typename XT>
struct Slot {
  int E0, E1, q0, q1;  // level's entry range and row range (block-relative positions)
  int col[kKP];
  VT val[kKP];
  XT xr[kKP];  // values from other blocks (possibly still the sentinel)
  int row;     // the first-pass row of this lane's group
  XT fv, bv;
  VT dg;
};

template <int OP, int TB, typename VT, typename XT>
__global__ __launch_bounds__(kNT) void tri_sweep_kernel(SweepDev sw, SweepPackDev pk, const XT* __restrict__ f,
                                                        XT* x, const XT* __restrict__ base, XT* __restrict__ out,
                                                        SweepSync sy, const int* __restrict__ done,
                                                        long spin_limit) {
  constexpr bool FWD = (OP == SWEEP_LOWER || OP == SWEEP_UNIT_LOWER);
  constexpr bool UNIT = (OP == SWEEP_UNIT_LOWER);
  constexpr bool OUT = (OP == SWEEP_UPPER_OUT);
  constexpr int NG = kNT / TB;
  extern __shared__ unsigned char smem_raw[];
  double* prod = reinterpret_cast<double*>(smem_raw);
  XT* xs = reinterpret_cast<XT*>(smem_raw + sw.off_xs);
  int* rows_l = reinterpret_cast<int*>(smem_raw + sw.off_rows);
  int* ptr_l = reinterpret_cast<int*>(smem_raw + sw.off_ptr);
  int* lvt = reinterpret_cast<int*>(smem_raw + sw.off_lvt);
  __shared__ int s_tick;
  __shared__ int s_last;
  if (done && *done) return;  // before taking a ticket: the counters stay untouched
  const int tid = threadIdx.x;
  const int g = tid / TB, lane = tid % TB;
  const VT* __restrict__ pval = reinterpret_cast<const VT*>(pk.val);
  const VT* __restrict__ pdiag = reinterpret_cast<const VT*>(pk.diag);

  for (;;) {
    if (tid == 0) s_tick = (int)atomicAdd(sy.ticket, 1u);
    __syncthreads();
    const int t = s_tick;
    __syncthreads();
    if (t >= sw.nblk) break;
    const int b = FWD ? t : sw.nblk - 1 - t;
    const int r0 = sw.blk_row[b], r1 = sw.blk_row[b + 1];
    const int nb = r1 - r0;
    const int lb = sw.blk_beg[b];
    const int nl = sw.blk_end[b] - lb;
    const int P0 = sw.lvl_ptr[lb];
    for (int q = tid; q <= nl; q += kNT) lvt[q] = sw.lvl_ptr[lb + q] - P0;
    for (int q = tid; q < nb; q += kNT) rows_l[q] = pk.row[P0 + q];
    for (int q = tid; q <= nb; q += kNT) ptr_l[q] = pk.ptr[P0 + q];
    __syncthreads();

    // loads of level m's entries and of the first-pass row data (addresses from LDS;
    // out-of-range lanes load a valid dummy address so that every step issues the same
    // number of loads)
    auto issue = [&](Slot<VT, XT>& s, int m) {
      int q0 = 0, q1 = 0, E0 = 0, E1 = 0;
      if (m < nl) {
        q0 = lvt[m];
        q1 = lvt[m + 1];
        E0 = ptr_l[q0];
        E1 = ptr_l[q1];
      }
      s.E0 = E0;
      s.E1 = E1;
      s.q0 = q0;
      s.q1 = q1;
#pragma unroll
      for (int k = 0; k < kKP; ++k) {
        const int e = E0 + tid + k * kNT;
        const int ec = e < E1 ? e : 0;
        s.col[k] = pk.col[ec];
        s.val[k] = pval[ec];
      }
      const int q = q0 + g;
      const int qc = q < q1 ? q : 0;
      s.row = rows_l[qc];
      s.fv = f[s.row];
      if (!UNIT) s.dg = pdiag[P0 + qc];
      if (OUT) s.bv = base[s.row];
    };
    // loads of the values a level reads from other blocks
    auto issue_remote = [&](Slot<VT, XT>& s) {
#pragma unroll
      for (int k = 0; k < kKP; ++k) {
        const int e = s.E0 + tid + k * kNT;
        const int c = s.col[k];
        const int j = (e < s.E1 && c < 0) ? -(c + 1) : 0;
        s.xr[k] = __hip_atomic_load(x + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    };
    auto ready = [&](XT v, int j) -> double {
      long spins = 0;
      while (is_sentinel(v)) {
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(x + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (++spins > spin_limit) {
          atomicOr(sy.err, 1u);
          return 0.0;
        }
        if ((spins & 255) == 0 && __hip_atomic_load(sy.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          return 0.0;
      }
      return (double)v;
    };
    auto finish = [&](int i, double sum, double fv, double dg, double bv) {
      const double xi = UNIT ? fv - sum : (fv - sum) / dg;
      const XT xo = (XT)xi;
      xs[i - r0] = xo;
      __hip_atomic_store(x + i, xo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (OUT) out[i] = (XT)(bv + (double)xo);
    };
    auto consume = [&](const Slot<VT, XT>& s) {
      const int E0 = s.E0, E1 = s.E1;
      const bool lng = (E1 - E0) > sw.pcap;  // a level of one row longer than the product slots
      double part = 0.0;
#pragma unroll
      for (int k = 0; k < kKP; ++k) {
        const int e = E0 + tid + k * kNT;
        if (e < E1) {
          const int c = s.col[k];
          const double xv = c >= 0 ? (double)xs[c] : ready(s.xr[k], -(c + 1));
          const double pr = (double)s.val[k] * xv;
          if (lng) part += pr;
          else prod[e - E0] = pr;
        }
      }
      for (int e = E0 + tid + kKP * kNT; e < E1; e += kNT) {
        const int c = pk.col[e];
        double xv;
        if (c >= 0) xv = (double)xs[c];
        else xv = ready(__hip_atomic_load(x + (-(c + 1)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), -(c + 1));
        const double pr = (double)pval[e] * xv;
        if (lng) part += pr;
        else prod[e - E0] = pr;
      }
      if (lng) prod[tid] = part;
      __syncthreads();
      if (lng) {
        if (g == 0) {
          double acc = 0.0;
          for (int j = lane; j < kNT; j += TB) acc += prod[j];
          acc = gsum<TB>(acc);
          if (lane == 0) finish(s.row, acc, (double)s.fv, UNIT ? 1.0 : (double)s.dg, OUT ? (double)s.bv : 0.0);
        }
      } else {
        // first pass: the rows whose data were prefetched
        const int q = s.q0 + g;
        if (q < s.q1) {
          const int a = ptr_l[q] - E0, len = ptr_l[q + 1] - ptr_l[q];
          double acc = 0.0;
          for (int j = lane; j < len; j += TB) acc += prod[a + j];
          acc = gsum<TB>(acc);
          if (lane == 0) finish(s.row, acc, (double)s.fv, UNIT ? 1.0 : (double)s.dg, OUT ? (double)s.bv : 0.0);
        }
        // levels with more rows than groups
        for (int q2 = q + NG; q2 < s.q1; q2 += NG) {
          const int a = ptr_l[q2] - E0, len = ptr_l[q2 + 1] - ptr_l[q2];
          double acc = 0.0;
          for (int j = lane; j < len; j += TB) acc += prod[a + j];
          acc = gsum<TB>(acc);
          if (lane == 0) {
            const int i = rows_l[q2];
            finish(i, acc, (double)f[i], UNIT ? 1.0 : (double)pdiag[P0 + q2], OUT ? (double)base[i] : 0.0);
          }
        }
      }
      __syncthreads();
    };
    // one level; then the other-block values of level m + 2 and the entries of m + 4
    auto step = [&](Slot<VT, XT>& s, Slot<VT, XT>& s2, int m) {
      consume(s);
      issue_remote(s2);
      issue(s, m + 4);
    };

    Slot<VT, XT> s0, s1, s2, s3;
    issue(s0, 0);
    issue(s1, 1);
    issue(s2, 2);
    issue(s3, 3);
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

template <int OP, int TB, typename VT, typename XT>
void launch_one(hipStream_t s, const SweepDev& sw, const SweepPackDev& pk, const void* f, void* x,
                const void* base, void* out, const SweepSync& sync, const int* done, long spin_limit) {
  static int attr = 65536;  // dynamic LDS the kernel may use without an attribute
  if (sw.lds > attr) {
    if (hipFuncSetAttribute((const void*)tri_sweep_kernel<OP, TB, VT, XT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kBudget) != hipSuccess) {
      (void)hipGetLastError();  // leave no sticky error; the launch below reports the failure
    } else {
      attr = kBudget;
    }
  }
  tri_sweep_kernel<OP, TB, VT, XT><<<sw.grid, kNT, sw.lds, s>>>(sw, pk, (const XT*)f, (XT*)x, (const XT*)base,
                                                                (XT*)out, sync, done, spin_limit);
}

template <int OP, typename VT, typename XT>
void dispatch_tb(hipStream_t s, const SweepDev& sw, const SweepPackDev& pk, const void* f, void* x,
                 const void* base, void* out, const SweepSync& sync, const int* done, long spin_limit) {
  switch (pk.tb) {
    case 1: launch_one<OP, 1, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    case 2: launch_one<OP, 2, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    case 4: launch_one<OP, 4, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    case 8: launch_one<OP, 8, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    case 16: launch_one<OP, 16, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    case 32: launch_one<OP, 32, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
    default: launch_one<OP, 64, VT, XT>(s, sw, pk, f, x, base, out, sync, done, spin_limit); break;
  }
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
  if (fp32) dispatch_tb<OPC, float, float>(s, sw, pk, f, x, base, out, sync, done, spin_limit);     \
  else dispatch_tb<OPC, double, double>(s, sw, pk, f, x, base, out, sync, done, spin_limit);
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
