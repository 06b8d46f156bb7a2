// Galerkin coarse matrices A_l = P_l^T A_{l+1} P_l (Section 3.2) on the GPU, as two
// sparse products C = X * Y: first A P, then R (A P) with R = P^T stored explicitly.
//
// Canonical order: entry (i, j) of C is accumulated from 0.0 by adding the rounded
// products x_ik * y_kj in increasing k (the column order of row i of X). One
// workgroup owns one output row at a time: it walks the row of X sequentially and,
// for each k, spreads the entries of row k of Y over its threads (distinct columns,
// so no two threads touch one accumulator in a step) with a barrier between steps.
// Accumulators live in an LDS hash table keyed by column. The row is then sorted by
// column and written out. This file is compiled without FMA contraction, so the
// result is bit-identical to any sequential evaluation in the same order.
#include <hip/hip_runtime.h>

#include <atomic>

#include "kernels.hpp"

namespace cpc {

namespace {

constexpr int kCap = 4096;  // distinct columns per output row held in LDS
constexpr int kNT = 256;

__device__ __forceinline__ unsigned slot_of(int j) { return ((unsigned)j * 2654435761u) & (kCap - 1); }

// returns the slot of column j, inserting it (value 0) when absent; -1 when full
__device__ __forceinline__ int find_or_insert(int* keys, double* vals, int j, bool with_vals, int* count) {
  unsigned h = slot_of(j);
  for (int probe = 0; probe < kCap; ++probe) {
    const int old = atomicCAS(&keys[h], -1, j);
    if (old == -1) {
      if (with_vals) vals[h] = 0.0;
      atomicAdd(count, 1);
      return (int)h;
    }
    if (old == j) return (int)h;
    h = (h + 1) & (kCap - 1);
  }
  return -1;
}

__global__ __launch_bounds__(kNT) void spgemm_count_kernel(int nrows, const int* __restrict__ xrp,
                                                           const int* __restrict__ xci, const int* __restrict__ yrp,
                                                           const int* __restrict__ yci, int* __restrict__ counts,
                                                           int* overflow) {
  extern __shared__ unsigned char smem[];
  int* keys = reinterpret_cast<int*>(smem);
  __shared__ int s_cnt;
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  for (int row = blockIdx.x; row < nrows; row += gridDim.x) {
    for (int t = tid; t < kCap; t += kNT) keys[t] = -1;
    if (tid == 0) {
      s_cnt = 0;
      s_bad = 0;
    }
    __syncthreads();
    for (int p = xrp[row]; p < xrp[row + 1]; ++p) {
      const int k = xci[p];
      for (int q = yrp[k] + tid; q < yrp[k + 1]; q += kNT) {
        if (find_or_insert(keys, nullptr, yci[q], false, &s_cnt) < 0) s_bad = 1;
      }
    }
    __syncthreads();
    if (tid == 0) {
      const bool wide = s_bad || s_cnt >= kCap;
      counts[row] = wide ? -1 : s_cnt;
      if (wide) atomicExch(overflow, 1);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kNT) void spgemm_fill_kernel(int nrows, const int* __restrict__ xrp,
                                                          const int* __restrict__ xci, const double* __restrict__ xv,
                                                          const int* __restrict__ yrp, const int* __restrict__ yci,
                                                          const double* __restrict__ yv, const int* __restrict__ crp,
                                                          int* __restrict__ cci, double* __restrict__ cv,
                                                          int* overflow) {
  extern __shared__ unsigned char smem[];
  double* vals = reinterpret_cast<double*>(smem);
  double* cvals = vals + kCap;
  int* keys = reinterpret_cast<int*>(cvals + kCap);
  int* ckeys = keys + kCap;
  __shared__ int s_cnt;
  __shared__ int s_bad;
  __shared__ int s_pos;
  const int tid = threadIdx.x;
  for (int row = blockIdx.x; row < nrows; row += gridDim.x) {
    if (crp[row + 1] - crp[row] >= kCap) continue;  // a wide row (uniform across the workgroup)
    for (int t = tid; t < kCap; t += kNT) keys[t] = -1;
    if (tid == 0) {
      s_cnt = 0;
      s_bad = 0;
      s_pos = 0;
    }
    __syncthreads();
    for (int p = xrp[row]; p < xrp[row + 1]; ++p) {
      const int k = xci[p];
      const double xk = xv[p];
      for (int q = yrp[k] + tid; q < yrp[k + 1]; q += kNT) {
        const int h = find_or_insert(keys, vals, yci[q], true, &s_cnt);
        if (h < 0) {
          s_bad = 1;
          continue;
        }
        const double prod = xk * yv[q];
        vals[h] = vals[h] + prod;
      }
      __syncthreads();  // orders the additions of step p before those of step p+1
    }
    // compact, then place each entry at its rank among the row's columns
    for (int t = tid; t < kCap; t += kNT) {
      if (keys[t] >= 0) {
        const int e = atomicAdd(&s_pos, 1);
        ckeys[e] = keys[t];
        cvals[e] = vals[t];
      }
    }
    __syncthreads();
    const int cnt = s_pos;
    const int base = crp[row];
    if (s_bad || cnt != crp[row + 1] - base) {
      if (tid == 0) atomicExch(overflow, 1);
    } else {
      for (int e = tid; e < cnt; e += kNT) {
        const int key = ckeys[e];
        int rank = 0;
        for (int f = 0; f < cnt; ++f) rank += (ckeys[f] < key);
        cci[base + rank] = key;
        cv[base + rank] = cvals[e];
      }
    }
    __syncthreads();
  }
}

// Wide rows: one workgroup per listed row at a time, with a slice of ncols entries of a
// device-memory marker (the tag row + 1 marks the row's columns; tags never repeat
// within a call, so the slice is zeroed once per call).
__global__ __launch_bounds__(kNT) void spgemm_count_wide_kernel(int nlist, const int* __restrict__ rows,
                                                                const int* __restrict__ xrp,
                                                                const int* __restrict__ xci,
                                                                const int* __restrict__ yrp,
                                                                const int* __restrict__ yci, int ncols, int* mark,
                                                                int* __restrict__ counts) {
  __shared__ int s_cnt;
  int* mk = mark + (size_t)blockIdx.x * ncols;
  const int tid = threadIdx.x;
  for (int li = blockIdx.x; li < nlist; li += gridDim.x) {
    const int row = rows[li], tag = row + 1;
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    int mine = 0;
    for (int p = xrp[row]; p < xrp[row + 1]; ++p) {
      const int k = xci[p];
      for (int q = yrp[k] + tid; q < yrp[k + 1]; q += kNT)
        if (atomicExch(&mk[yci[q]], tag) != tag) ++mine;  // the first to mark a column counts it
    }
    atomicAdd(&s_cnt, mine);
    __syncthreads();
    if (tid == 0) counts[row] = s_cnt;
    __syncthreads();
  }
}

// Numeric pass of the wide rows: a dense accumulator slice per workgroup. Step p adds
// x_ik * y_kj for the entries of row k = X(i, p) (distinct columns, one thread each),
// with a barrier between steps: the order of each entry's additions is that of the LDS
// table kernel. The row is then written in increasing column by a scan of the marker.
__global__ __launch_bounds__(kNT) void spgemm_fill_wide_kernel(int nlist, const int* __restrict__ rows,
                                                               const int* __restrict__ xrp,
                                                               const int* __restrict__ xci,
                                                               const double* __restrict__ xv,
                                                               const int* __restrict__ yrp,
                                                               const int* __restrict__ yci,
                                                               const double* __restrict__ yv, int ncols, int* mark,
                                                               double* acc, const int* __restrict__ crp,
                                                               int* __restrict__ cci, double* __restrict__ cv,
                                                               int* overflow) {
  __shared__ int s_scan[kNT];
  __shared__ int s_base;
  int* mk = mark + (size_t)blockIdx.x * ncols;
  double* ac = acc + (size_t)blockIdx.x * ncols;
  const int tid = threadIdx.x;
  for (int li = blockIdx.x; li < nlist; li += gridDim.x) {
    const int row = rows[li], tag = row + 1;
    for (int p = xrp[row]; p < xrp[row + 1]; ++p) {
      const int k = xci[p];
      const double xk = xv[p];
      for (int q = yrp[k] + tid; q < yrp[k + 1]; q += kNT) {
        const int j = yci[q];
        const double prod = xk * yv[q];
        if (mk[j] != tag) {
          mk[j] = tag;
          ac[j] = 0.0;
        }
        ac[j] = ac[j] + prod;
      }
      __syncthreads();  // orders the additions of step p before those of step p+1
    }
    if (tid == 0) s_base = 0;
    __syncthreads();
    const int base = crp[row], cnt = crp[row + 1] - base;
    for (int c0 = 0; c0 < ncols; c0 += kNT) {
      const int j = c0 + tid;
      const int f = (j < ncols && mk[j] == tag) ? 1 : 0;
      s_scan[tid] = f;
      __syncthreads();
      for (int o = 1; o < kNT; o <<= 1) {  // inclusive scan of the chunk's flags
        const int v = tid >= o ? s_scan[tid - o] : 0;
        __syncthreads();
        s_scan[tid] += v;
        __syncthreads();
      }
      const int pos = s_base + s_scan[tid] - f;
      if (f && pos < cnt) {
        cci[base + pos] = j;
        cv[base + pos] = ac[j];
      }
      __syncthreads();
      if (tid == kNT - 1) s_base += s_scan[tid];
      __syncthreads();
    }
    if (tid == 0 && s_base != cnt) atomicExch(overflow, 1);
    __syncthreads();
  }
}

}  // namespace

int spgemm_table_capacity() { return kCap; }

void launch_spgemm_count(hipStream_t s, int nrows, const int* xrp, const int* xci, const int* yrp, const int* yci,
                         int* counts, int* wide) {
  if (nrows <= 0) return;
  const size_t lds = sizeof(int) * kCap;
  const int grid = nrows < 4096 ? nrows : 4096;
  spgemm_count_kernel<<<grid, kNT, lds, s>>>(nrows, xrp, xci, yrp, yci, counts, wide);
}

void launch_spgemm_count_wide(hipStream_t s, int nlist, const int* rows, const int* xrp, const int* xci,
                              const int* yrp, const int* yci, int ncols, int* mark, int nwg, int* counts) {
  if (nlist <= 0 || nwg <= 0) return;
  spgemm_count_wide_kernel<<<nwg, kNT, 0, s>>>(nlist, rows, xrp, xci, yrp, yci, ncols, mark, counts);
}

void launch_spgemm_fill_wide(hipStream_t s, int nlist, const int* rows, const int* xrp, const int* xci,
                             const double* xv, const int* yrp, const int* yci, const double* yv, int ncols, int* mark,
                             double* acc, int nwg, const int* crp, int* cci, double* cv, int* overflow) {
  if (nlist <= 0 || nwg <= 0) return;
  spgemm_fill_wide_kernel<<<nwg, kNT, 0, s>>>(nlist, rows, xrp, xci, xv, yrp, yci, yv, ncols, mark, acc, crp, cci,
                                               cv, overflow);
}

void launch_spgemm_fill(hipStream_t s, int nrows, const int* xrp, const int* xci, const double* xv, const int* yrp,
                        const int* yci, const double* yv, const int* crp, int* cci, double* cv, int* overflow) {
  if (nrows <= 0) return;
  const size_t lds = (sizeof(double) * 2 + sizeof(int) * 2) * kCap;
  static std::atomic<bool> attr_set{false};  // batch setups launch from several host threads
  if (!attr_set.load()) {
    if (hipFuncSetAttribute((const void*)spgemm_fill_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) ==
        hipSuccess)
      attr_set.store(true);
    else
      (void)hipGetLastError();
  }
  const int grid = nrows < 2048 ? nrows : 2048;
  spgemm_fill_kernel<<<grid, kNT, lds, s>>>(nrows, xrp, xci, xv, yrp, yci, yv, crp, cci, cv, overflow);
}

}  // namespace cpc
