// Persistent, block-pipelined, level-scheduled triangular sweep with prefetched
// row data (forward/backward Gauss-Seidel, ILU(0) L and U solves).
//
// Each sweep has a packed copy of the rows it touches, in processing order: the
// p-th processed row is row[p], its dependency-side entries are col/val[ptr[p] ..
// ptr[p+1]) in column order, its diagonal is diag[p]. A workgroup (4 waves) takes
// blocks of contiguous rows from a ticket counter in dependency order and stages
// the block's level table, row list and entry offsets in LDS.
//
// Waves 1-3 are workers: groups of TPR lanes solve the rows of one level set per
// step and keep the block's solved values in LDS only. Row data are prefetched
// kDepth levels ahead into a ring of register slots. Their addresses come from LDS,
// not from loads still in flight, because the vector-memory counter completes in
// order: a dependent load chain would drain every younger prefetch. The in-place
// backward sweep also needs the pre-sweep values of a row's lower neighbours; those
// are gathered one level ahead.
//
// Wave 0 is the coordinator. It waits on other blocks' progress counters. After
// levels another block waits for, and at the end of the block, it copies the rows
// solved since its last copy from LDS to the global vector with agent-scope
// (write-through) stores, waits for their completion, and then advances the block's
// progress counter. Readers of another block's rows use agent-scope loads. No
// cache-wide release/acquire fences are used: with hundreds of workgroups
// synchronising every level, L2-wide write-backs and invalidations would dominate.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cpc {

namespace {

constexpr int kNT = 256;        // threads per workgroup
constexpr int kWorkers = 192;   // waves 1-3
constexpr int kK = 4;           // entries per lane held in a prefetch slot
constexpr int kLvCap = 4096;    // block level-table entries staged in LDS

template <int W>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

template <typename VT, typename XT>
struct Slot {
  int row, e0, e1;
  VT diag;
  int col[kK];
  VT val[kK];
  XT fv, bv;
  XT xo[kK];  // pre-sweep values of lower neighbours (in-place backward sweep)
};

template <int OP, int TPR, typename VT, typename XT>
__global__ __launch_bounds__(kNT) void sweep_kernel5(SweepDev sw, SweepPackDev pk, int n, const XT* __restrict__ f,
                                                     XT* x, const XT* __restrict__ base, XT* __restrict__ out,
                                                     SweepSync sy, const int* __restrict__ done, long spin_limit) {
  constexpr bool FWD = (OP == SWEEP_FGS0 || OP == SWEEP_ILU_L);
  constexpr bool BGS = (OP == SWEEP_BGS_IP);
  constexpr int NGRP = kWorkers / TPR;
  extern __shared__ unsigned char smem_raw[];
  XT* xs = reinterpret_cast<XT*>(smem_raw);
  int* rows_l = reinterpret_cast<int*>(smem_raw + ((sw.R * (int)sizeof(XT) + 15) & ~15));
  int* ptr_l = rows_l + ((sw.R + 3) & ~3);
  int* lvt = ptr_l + ((sw.R + 4) & ~3);
  __shared__ int s_tick;
  __shared__ int s_last;
  if (done && *done) return;  // before taking a ticket: the counters stay untouched
  const int tid = threadIdx.x;
  const bool coord = tid < 64;
  const int wt = tid - 64;
  const int lane = coord ? 0 : wt % TPR;
  const int grp = coord ? 0 : wt / TPR;
  const VT* __restrict__ pval = reinterpret_cast<const VT*>(pk.val);
  const VT* __restrict__ pdiag = reinterpret_cast<const VT*>(pk.diag);

  for (;;) {
    if (tid == 0) s_tick = (int)atomicAdd(sy.ticket, 1u);
    __syncthreads();
    const int t = s_tick;
    __syncthreads();
    if (t >= sw.nblk) break;
    const int b = FWD ? t : sw.nblk - 1 - t;
    const int r0 = sw.blk_row[b];
    const int r1 = sw.blk_row[b + 1];
    const int nb = r1 - r0;
    const int lb = sw.blk_beg[b], le = sw.blk_end[b];
    const int nl = le - lb;
    const int P0 = sw.lvl_ptr[lb];
    for (int q = tid; q <= nl && q <= kLvCap; q += kNT) lvt[q] = sw.lvl_ptr[lb + q] - P0;
    for (int q = tid; q < nb; q += kNT) rows_l[q] = pk.row[P0 + q];
    for (int q = tid; q <= nb; q += kNT) ptr_l[q] = pk.ptr[P0 + q];
    __syncthreads();
    int copied = 0;  // rows (processing order within the block) already copied out

    auto LP = [&](int m) -> int { return m <= kLvCap ? lvt[m] : sw.lvl_ptr[lb + m] - P0; };
    // issue the loads of this group's first row of level m (addresses from LDS)
    auto issue = [&](Slot<VT, XT>& s, int m) {
      s.row = -1;
      if (coord || m >= nl) return;
      const int q = LP(m) + grp;
      if (q >= LP(m + 1)) return;
      s.row = rows_l[q];
      s.e0 = ptr_l[q];
      s.e1 = ptr_l[q + 1];
      if (OP != SWEEP_ILU_L) s.diag = pdiag[P0 + q];
#pragma unroll
      for (int k = 0; k < kK; ++k) {
        const int e = s.e0 + lane + k * TPR;
        s.col[k] = -1;
        if (e < s.e1) {
          s.col[k] = pk.col[e];
          s.val[k] = pval[e];
        }
      }
      if (lane == 0) {
        s.fv = f[s.row];
        if (OP == SWEEP_ILU_U && out) s.bv = base[s.row];
      }
    };
    // in-place backward sweep: pre-sweep values of the row's lower neighbours
    auto gather_old = [&](Slot<VT, XT>& s) {
      if (!BGS || coord || s.row < 0) return;
#pragma unroll
      for (int k = 0; k < kK; ++k)
        if (s.col[k] >= 0 && s.col[k] < s.row) s.xo[k] = x[s.col[k]];
    };
    auto xnew = [&](int j) -> double {
      // solved in this block: LDS; solved by an earlier block: agent-scope load
      const bool local = FWD ? (j >= r0) : (j < r1);
      if (local) return (double)xs[j - r0];
      return (double)__hip_atomic_load(x + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    auto xval = [&](int j, int i) -> double {
      if (BGS && j < i) return (double)x[j];  // value from before the sweep
      return xnew(j);
    };
    auto finish = [&](int i, double s, double fv, double diag, double bv) {
      double xi;
      if (OP == SWEEP_ILU_L) xi = fv - s;
      else xi = (fv - s) / diag;
      const XT xo = (XT)xi;
      xs[i - r0] = xo;
      if (OP == SWEEP_ILU_U && out) out[i] = (XT)(bv + (double)xo);
    };
    auto consume = [&](const Slot<VT, XT>& s, int m) {
      if (s.row >= 0) {
        const int i = s.row;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kK; ++k) {
          if (s.col[k] < 0) continue;
          const double xj = (BGS && s.col[k] < i) ? (double)s.xo[k] : xnew(s.col[k]);
          acc += (double)s.val[k] * xj;
        }
        for (int e = s.e0 + lane + kK * TPR; e < s.e1; e += TPR) acc += (double)pval[e] * xval(pk.col[e], i);
        acc = gsum<TPR>(acc);
        if (lane == 0)
          finish(i, acc, (double)s.fv, OP == SWEEP_ILU_L ? 1.0 : (double)s.diag,
                 OP == SWEEP_ILU_U ? (double)s.bv : 0.0);
      }
      // rows beyond the first NGRP of this level (not prefetched)
      const int q1 = LP(m + 1);
      for (int q = LP(m) + grp + NGRP; q < q1; q += NGRP) {
        const int i = rows_l[q];
        double acc = 0.0;
        for (int e = ptr_l[q] + lane; e < ptr_l[q + 1]; e += TPR) acc += (double)pval[e] * xval(pk.col[e], i);
        acc = gsum<TPR>(acc);
        if (lane == 0)
          finish(i, acc, (double)f[i], OP == SWEEP_ILU_L ? 1.0 : (double)pdiag[P0 + q],
                 (OP == SWEEP_ILU_U && out) ? (double)base[i] : 0.0);
      }
    };
    auto wait_level = [&](int lv) {
      const int w0 = sw.wait_ptr[lv], w1 = sw.wait_ptr[lv + 1];
      for (int w = w0 + tid; w < w1; w += 64) {
        const unsigned need = (unsigned)sw.wait_need[w];
        unsigned* pp = sy.progress + sw.wait_blk[w];
        long spins = 0;
        while (__hip_atomic_load(pp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > spin_limit) {
            atomicOr(sy.err, 1u);
            break;
          }
          if ((spins & 1023) == 0 && __hip_atomic_load(sy.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        }
      }
      asm volatile("" ::: "memory");
    };
    // copy rows solved up to level m to the global vector, wait for the stores to
    // complete, then publish progress m + 1
    auto publish = [&](int m, bool advance) {
      const int upto = LP(m + 1);
      for (int q = copied + tid; q < upto; q += 64) {
        const int i = rows_l[q];
        __hip_atomic_store(x + i, xs[i - r0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      copied = upto;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      if (advance && tid == 0)
        __hip_atomic_store(sy.progress + b, (unsigned)(m + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // one level: wait, solve, publish; then refill this slot four levels ahead and
    // gather the pre-sweep neighbour values of the next slot
    auto step = [&](Slot<VT, XT>& s, Slot<VT, XT>& next, int m) {
      const int lv = lb + m;
      if (coord) wait_level(lv);
      else gather_old(next);
      __syncthreads();
      if (!coord) consume(s, m);
      __syncthreads();
      if (coord && (sw.publish[lv] || m + 1 == nl)) publish(m, sw.publish[lv] != 0);
      issue(s, m + 4);
    };

    Slot<VT, XT> s0, s1, s2, s3;
    issue(s0, 0);
    issue(s1, 1);
    issue(s2, 2);
    issue(s3, 3);
    gather_old(s0);
    for (int m = 0; m < nl; m += 4) {
      step(s0, s1, m);
      if (m + 1 < nl) step(s1, s2, m + 1);
      if (m + 2 < nl) step(s2, s3, m + 2);
      if (m + 3 < nl) step(s3, s0, m + 3);
    }
    __syncthreads();  // the coordinator's final copy reads LDS the next block overwrites
  }
  if (tid == 0) s_last = (atomicAdd(sy.exited, 1u) == gridDim.x - 1);
  __syncthreads();
  if (s_last) {
    __threadfence();
    for (int i = tid; i < sw.nblk; i += kNT) sy.progress[i] = 0u;
    if (tid == 0) {
      *sy.ticket = 0u;
      *sy.exited = 0u;
    }
  }
}

template <int OP, int TPR, typename VT, typename XT>
void launch_one(hipStream_t s, const SweepDev& sw, const SweepPackDev& pk, int n, const void* f, void* x,
                const void* base, void* out, const SweepSync& sync, const int* done, long spin_limit) {
  const size_t lds = (size_t)((sw.R * sizeof(XT) + 15) & ~size_t(15)) + sizeof(int) * ((sw.R + 3) & ~3) +
                     sizeof(int) * ((sw.R + 4) & ~3) + sizeof(int) * (kLvCap + 1);
  static size_t attr = 65536;  // dynamic LDS the kernel may use without an attribute
  if (lds > attr) {
    if (hipFuncSetAttribute((const void*)sweep_kernel5<OP, TPR, VT, XT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess) {
      (void)hipGetLastError();  // leave no sticky error; the launch below reports the failure
    } else {
      attr = lds;
    }
  }
  sweep_kernel5<OP, TPR, VT, XT><<<sw.grid, kNT, lds, s>>>(sw, pk, n, (const XT*)f, (XT*)x, (const XT*)base,
                                                          (XT*)out, sync, done, spin_limit);
}

template <int OP, typename VT, typename XT>
void dispatch_tpr(hipStream_t s, const SweepDev& sw, const SweepPackDev& pk, int n, const void* f, void* x,
                  const void* base, void* out, const SweepSync& sync, const int* done, long spin_limit) {
  switch (sw.tpr) {
    case 1: launch_one<OP, 1, VT, XT>(s, sw, pk, n, f, x, base, out, sync, done, spin_limit); break;
    case 2: launch_one<OP, 2, VT, XT>(s, sw, pk, n, f, x, base, out, sync, done, spin_limit); break;
    case 4: launch_one<OP, 4, VT, XT>(s, sw, pk, n, f, x, base, out, sync, done, spin_limit); break;
    case 8: launch_one<OP, 8, VT, XT>(s, sw, pk, n, f, x, base, out, sync, done, spin_limit); break;
    case 16: launch_one<OP, 16, VT, XT>(s, sw, pk, n, f, x, base, out, sync, done, spin_limit); break;
    case 32: launch_one<OP, 32, VT, XT>(s, sw, pk, n, f, x, base, out, sync, done, spin_limit); break;
    default: launch_one<OP, 64, VT, XT>(s, sw, pk, n, f, x, base, out, sync, done, spin_limit); break;
  }
}

}  // namespace

int sweep_max_rows_per_block() { return 8192; }
int sweep_entries_per_lane() { return kK; }

void launch_sweep_packed(hipStream_t s, int op, const SweepDev& sw, const SweepPackDev& pk, int n, bool fp32,
                         const void* f, void* x, const void* base, void* out, const SweepSync& sync,
                         const int* done, long spin_limit) {
  if (sw.n <= 0) return;
#define CPC_SW(OPC)                                                                                        \
  if (fp32) dispatch_tpr<OPC, float, float>(s, sw, pk, n, f, x, base, out, sync, done, spin_limit);     \
  else dispatch_tpr<OPC, double, double>(s, sw, pk, n, f, x, base, out, sync, done, spin_limit);
  switch (op) {
    case SWEEP_FGS0: CPC_SW(SWEEP_FGS0) break;
    case SWEEP_BGS_IP: CPC_SW(SWEEP_BGS_IP) break;
    case SWEEP_ILU_L: CPC_SW(SWEEP_ILU_L) break;
    default: CPC_SW(SWEEP_ILU_U) break;
  }
#undef CPC_SW
}

}  // namespace cpc
