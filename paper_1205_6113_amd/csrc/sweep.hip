// Persistent, block-pipelined, level-scheduled triangular sweep with prefetched
// row data (forward/backward Gauss-Seidel, ILU(0) L and U solves).
//
// Each sweep has a packed copy of the rows it touches, in processing order: the
// p-th processed row is row[p], its dependency-side entries are col/val[ptr[p] ..
// ptr[p+1]) in column order, its diagonal is diag[p]. A workgroup (4 waves) takes
// blocks of contiguous rows from a ticket counter in dependency order. Waves 1-3
// are workers: groups of TPR lanes solve the rows of one level set per step and
// keep the block's solved values in LDS only. The row data of the next level
// (entries into registers) and of the level after (row index, entry range,
// diagonal) are loaded before the current level's wait and barrier, so their HBM
// latency overlaps the synchronisation instead of sitting on the dependency chain.
// Wave 0 is the coordinator. It waits on other blocks' progress counters, and
// after levels another block waits for (and at the end of the block) it copies the
// rows solved since its last copy from LDS to the global vector with agent-scope
// (write-through) stores, waits for their completion, and then advances the block's
// progress counter. Readers of another block's rows use agent-scope loads. No
// cache-wide release/acquire fences are used: with hundreds of workgroups
// synchronising every level, L2-wide write-backs and invalidations would dominate.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cpc {

namespace {

constexpr int kNT = 256;     // threads per workgroup
constexpr int kWorkers = 192;  // waves 1-3
constexpr int kK = 8;        // entries per lane held in registers
constexpr int kLvCap = 4096; // block level-table entries staged in LDS

template <int W>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

template <typename VT>
struct Meta {
  int row, e0, e1;
  VT diag;
};

template <typename VT, typename XT>
struct Ent {
  int col[kK];
  VT val[kK];
  XT fv, bv;
};

template <int OP, int TPR, typename VT, typename XT>
__global__ __launch_bounds__(kNT) void sweep3_kernel(SweepDev sw, SweepPackDev pk, int n, const XT* __restrict__ f,
                                                     XT* x, const XT* __restrict__ base, XT* __restrict__ out,
                                                     SweepSync sy, const int* __restrict__ done, long spin_limit) {
  constexpr bool FWD = (OP == SWEEP_FGS0 || OP == SWEEP_ILU_L);
  constexpr int NGRP = kWorkers / TPR;
  extern __shared__ unsigned char smem_raw[];
  XT* xs = reinterpret_cast<XT*>(smem_raw);
  int* rows_l = reinterpret_cast<int*>(smem_raw + ((sw.R * (int)sizeof(XT) + 15) & ~15));
  int* lvt = rows_l + ((sw.R + 3) & ~3);
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
    const int r0 = b * sw.R;
    const int r1 = min(n, r0 + sw.R);
    const int lb = sw.blk_beg[b], le = sw.blk_end[b];
    const int nl = le - lb;
    for (int q = tid; q <= nl && q <= kLvCap; q += kNT) lvt[q] = sw.lvl_ptr[lb + q];
    const int P0 = sw.lvl_ptr[lb];
    for (int q = tid; q < r1 - r0; q += kNT) rows_l[q] = pk.row[P0 + q];
    __syncthreads();
    int copied = 0;  // rows (in processing order) already copied to the global vector
    auto LP = [&](int m) -> int { return m <= kLvCap ? lvt[m] : sw.lvl_ptr[lb + m]; };
    auto load_meta = [&](int m, Meta<VT>& mt) {
      mt.row = -1;
      if (m < nl) {
        const int p = LP(m) + grp;
        if (p < LP(m + 1)) {
          mt.row = pk.row[p];
          mt.e0 = pk.ptr[p];
          mt.e1 = pk.ptr[p + 1];
          if (OP != SWEEP_ILU_L) mt.diag = pdiag[p];
        }
      }
    };
    auto load_ent = [&](const Meta<VT>& mt, Ent<VT, XT>& en) {
#pragma unroll
      for (int k = 0; k < kK; ++k) en.col[k] = -1;
      if (mt.row >= 0) {
#pragma unroll
        for (int k = 0; k < kK; ++k) {
          const int e = mt.e0 + lane + k * TPR;
          if (e < mt.e1) {
            en.col[k] = pk.col[e];
            en.val[k] = pval[e];
          }
        }
        if (lane == 0) {
          en.fv = f[mt.row];
          if (OP == SWEEP_ILU_U && out) en.bv = base[mt.row];
        }
      }
    };
    auto xval = [&](int j, int i) -> double {
      // solved in this block: LDS; solved by an earlier block: agent-scope load;
      // in-place backward sweep, j < i: the value from before the sweep
      if (OP == SWEEP_FGS0 || OP == SWEEP_ILU_L) {
        if (j >= r0) return (double)xs[j - r0];
        return (double)__hip_atomic_load(x + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (OP == SWEEP_ILU_U) {
        if (j < r1) return (double)xs[j - r0];
        return (double)__hip_atomic_load(x + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        if (j < i) return (double)x[j];
        if (j < r1) return (double)xs[j - r0];
        return (double)__hip_atomic_load(x + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    };
    auto finish = [&](int i, double s, double fv, double diag, double bv) {
      double xi;
      if (OP == SWEEP_ILU_L) xi = fv - s;
      else xi = (fv - s) / diag;
      const XT xo = (XT)xi;
      xs[i - r0] = xo;
      if (OP == SWEEP_ILU_U && out) out[i] = (XT)(bv + (double)xo);
    };
    // coordinator: copy rows solved up to level m (processing order) to the global
    // vector, wait for the stores to complete, then publish progress m + 1
    auto publish = [&](int m, bool advance) {
      const int upto = LP(m + 1) - P0;
      for (int q = copied + tid; q < upto; q += 64) {
        const int i = rows_l[q];
        __hip_atomic_store(x + i, xs[i - r0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      copied = upto;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      if (advance && tid == 0)
        __hip_atomic_store(sy.progress + b, (unsigned)(m + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };

    Meta<VT> ma, mb;
    Ent<VT, XT> ea;
    if (!coord) {
      load_meta(0, ma);
      load_meta(1, mb);
      load_ent(ma, ea);
    }
    for (int m = 0; m < nl; ++m) {
      const int lv = lb + m;
      Meta<VT> mc;
      Ent<VT, XT> eb;
      if (!coord) {
        load_ent(mb, eb);     // entries of the next level
        load_meta(m + 2, mc); // row data of the level after
      } else {
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
        // the workers' agent-scope loads are issued after this barrier, i.e. after
        // the counters showed the producers' stores complete
        asm volatile("" ::: "memory");
      }
      __syncthreads();
      if (!coord) {
        const int p0 = LP(m), p1 = LP(m + 1);
        if (ma.row >= 0) {
          const int i = ma.row;
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < kK; ++k)
            if (ea.col[k] >= 0) s += (double)ea.val[k] * xval(ea.col[k], i);
          for (int e = ma.e0 + lane + kK * TPR; e < ma.e1; e += TPR) s += (double)pval[e] * xval(pk.col[e], i);
          s = gsum<TPR>(s);
          if (lane == 0)
            finish(i, s, (double)ea.fv, OP == SWEEP_ILU_L ? 1.0 : (double)ma.diag,
                   OP == SWEEP_ILU_U ? (double)ea.bv : 0.0);
        }
        // rows beyond the first NGRP of this level (not prefetched)
        for (int p = p0 + grp + NGRP; p < p1; p += NGRP) {
          const int i = pk.row[p];
          const int e0 = pk.ptr[p], e1 = pk.ptr[p + 1];
          double s = 0.0;
          for (int e = e0 + lane; e < e1; e += TPR) s += (double)pval[e] * xval(pk.col[e], i);
          s = gsum<TPR>(s);
          if (lane == 0)
            finish(i, s, (double)f[i], OP == SWEEP_ILU_L ? 1.0 : (double)pdiag[p],
                   (OP == SWEEP_ILU_U && out) ? (double)base[i] : 0.0);
        }
      }
      __syncthreads();
      if (coord && (sw.publish[lv] || m + 1 == nl)) publish(m, sw.publish[lv] != 0);
      if (!coord) {
        ma = mb;
        ea = eb;
        mb = mc;
      }
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
                     sizeof(int) * (kLvCap + 1);
  static size_t attr = 65536;  // dynamic LDS the kernel may use without an attribute
  if (lds > attr) {
    if (hipFuncSetAttribute((const void*)sweep3_kernel<OP, TPR, VT, XT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess) {
      (void)hipGetLastError();  // leave no sticky error; the launch below reports the failure
    } else {
      attr = lds;
    }
  }
  sweep3_kernel<OP, TPR, VT, XT><<<sw.grid, kNT, lds, s>>>(sw, pk, n, (const XT*)f, (XT*)x, (const XT*)base,
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
