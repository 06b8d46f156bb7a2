// HIP kernels of the SOLVE phase for gfx950 (wave64).
//
//  * CSR SpMV family with TPR lanes per row (TPR in {1,...,64}); rows are spread
//    over the grid, each group of TPR lanes reads its row's column/value streams
//    contiguously and reduces with cross-lane shuffles.
//  * Fused PCG vector kernels with a deterministic two-stage reduction: each
//    workgroup writes one partial, the last workgroup to arrive sums the
//    partials in index order and updates the scalars (alpha, beta, relres,
//    convergence flag) on the device.
//  * Dense coarsest-level matvec, elementwise vector kernels, FP64->FP32 copies.
//  The level-scheduled sweeps live in sweep.hip.
#include "kernels.hpp"
#include "csr_row.hpp"
#include "wave_sum.hpp"

#include <hip/hip_runtime.h>

namespace cpc {

namespace {

constexpr int kNT = 256;          // threads per workgroup for the streaming kernels
constexpr int kRedGrid = 1024;    // workgroups of the reduction kernels (grid-stride)
static_assert(2 * kRedGrid <= kPartials, "the initial residual's two reductions share the partials");

template <typename T>
__device__ __forceinline__ double ld(const T* p, long i) {
  return (double)p[i];
}

template <typename T>
__device__ __forceinline__ void st(T* p, long i, double v) {
  p[i] = (T)v;
}

// Sum over the workgroup (kNT threads). Fixed tree: deterministic.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = gsum<64>(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  }
  return s;  // valid in thread 0
}

// Last-workgroup reduction: every workgroup publishes its partial; the last one to
// arrive returns true in all of its threads and has the total in *total (thread 0).
__device__ bool arrive(double part, double* partials, unsigned* counter, double* sh, double* total) {
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = part;
    __threadfence();
    const unsigned t = atomicAdd(counter, 1u);
    s_last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  double s = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) s += __builtin_nontemporal_load(partials + i);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    *total = s;
    *counter = 0u;
  }
  return true;
}

// ----------------------------------------------------------------------------
// SpMV family


// rid (may be null): row k of the matrix is entry rid[k] of f and y (the rows of one
// step of the block substitution, which lie in several systems of a batch).
template <int TPR, int U, typename VT, typename XT, typename FT, typename YT>
__global__ __launch_bounds__(kNT) void spmv_kernel(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const VT* __restrict__ v, const XT* __restrict__ x,
                                                   const FT* __restrict__ f, YT* __restrict__ y, int mode,
                                                   const int* __restrict__ rid, SysMask mask,
                                                   const int* __restrict__ done) {
  constexpr int RPB = kNT / TPR;
  const int lane = threadIdx.x % TPR;
  const int stride = gridDim.x * RPB;
  int i = blockIdx.x * RPB + threadIdx.x / TPR;
  // A row's bounds and the term its product is combined with (f_i, or y_i when adding)
  // are read before they are needed: the first row's together with the convergence flag,
  // the next row's while this one is summed, so the flag and those reads add no step to
  // the chain of dependent loads (rows bounds, then entries, then x).
  int b = 0, e = 0, o = 0;
  double g = 0.0;
  if (i < n) {
    b = rp[i];
    e = rp[i + 1];
    o = rid ? rid[i] : i;
    g = mode == 1 ? ld(f, o) : (mode == 2 ? ld(y, o) : 0.0);
  }
  if (done && *done) return;
  for (; i < n; i += stride) {
    const bool skip = masked(mask, o);  // a row of a system that has stopped
    const double s0 = row_dot<TPR, U>(b + lane, skip ? b : e, ci, v, x);
    const int in = i + stride;
    const double gi = g;
    const int oi = o;
    if (in < n) {
      b = rp[in];
      e = rp[in + 1];
      o = rid ? rid[in] : in;
      g = mode == 1 ? ld(f, o) : (mode == 2 ? ld(y, o) : 0.0);
    }
    const double s = gsum<TPR>(s0);
    if (lane == 0 && !skip) {
      if (mode == 0) st(y, oi, s);
      else if (mode == 1) st(y, oi, gi - s);
      else st(y, oi, gi + s);
    }
  }
}

template <int TPR>
__global__ __launch_bounds__(kNT) void spmv_pq_kernel(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                      const double* __restrict__ v, const double* __restrict__ p,
                                                      double* __restrict__ q, double* partials, PcgState* stt) {
  __shared__ double sh[kNT / 64];
  if (stt->done) return;
  constexpr int RPB = kNT / TPR;
  const int lane = threadIdx.x % TPR;
  double acc = 0.0;
  for (int i = blockIdx.x * RPB + threadIdx.x / TPR; i < n; i += gridDim.x * RPB) {
    const int b = rp[i], e = rp[i + 1];
    double s = row_dot<TPR, 1>(b + lane, e, ci, v, p);
    s = gsum<TPR>(s);
    if (lane == 0) {
      q[i] = s;
      acc += s * p[i];
    }
  }
  double part = block_sum(acc, sh);
  double tot;
  if (arrive(part, partials, &stt->cnt[0], sh, &tot) && threadIdx.x == 0) {
    stt->pq = tot;
    if (!(tot > 0.0) || !isfinite(tot)) {
      stt->done = DONE_BREAKDOWN;
    } else {
      stt->alpha = stt->rz / tot;
    }
  }
}

__global__ __launch_bounds__(kNT) void update_xr_kernel(int n, double* __restrict__ x, double* __restrict__ r,
                                                        const double* __restrict__ p, const double* __restrict__ q,
                                                        double* partials, PcgState* stt) {
  __shared__ double sh[kNT / 64];
  if (stt->done) return;
  const double a = stt->alpha;
  double acc = 0.0;
  for (int i = blockIdx.x * kNT + threadIdx.x; i < n; i += gridDim.x * kNT) {
    x[i] = x[i] + a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  double part = block_sum(acc, sh);
  double tot;
  if (arrive(part, partials, &stt->cnt[1], sh, &tot) && threadIdx.x == 0) {
    stt->rr = tot;
    stt->iters += 1;
    const double rel = sqrt(tot) / sqrt(stt->bb);
    stt->relres = rel;
    if (!isfinite(rel)) stt->done = DONE_BREAKDOWN;
    else if (rel <= stt->tol) stt->done = DONE_CONVERGED;
    else if (stt->iters >= stt->maxit) stt->done = DONE_MAXIT;
  }
}

__global__ __launch_bounds__(kNT) void dot_rz_kernel(int n, const double* __restrict__ r, const double* __restrict__ z,
                                                     double* __restrict__ p, double* partials, PcgState* stt,
                                                     int first) {
  __shared__ double sh[kNT / 64];
  if (stt->done) return;
  double acc = 0.0;
  for (int i = blockIdx.x * kNT + threadIdx.x; i < n; i += gridDim.x * kNT) {
    const double zi = z[i];
    acc += r[i] * zi;
    if (first) p[i] = zi;
  }
  double part = block_sum(acc, sh);
  double tot;
  if (arrive(part, partials, &stt->cnt[2], sh, &tot) && threadIdx.x == 0) {
    if (!(tot > 0.0) || !isfinite(tot)) {
      stt->done = DONE_BREAKDOWN;
    } else {
      if (!first) stt->beta = tot / stt->rz;
      stt->rz = tot;
    }
  }
}

__global__ __launch_bounds__(kNT) void update_p_kernel(int n, const double* __restrict__ z, double* __restrict__ p,
                                                       const PcgState* stt) {
  if (stt->done) return;
  const double b = stt->beta;
  for (int i = blockIdx.x * kNT + threadIdx.x; i < n; i += gridDim.x * kNT) p[i] = z[i] + b * p[i];
}

template <int TPR>
__global__ __launch_bounds__(kNT) void pcg_init_kernel(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ v, const double* __restrict__ b,
                                                       double* __restrict__ x, double* __restrict__ r, int use_x0,
                                                       double* partials, PcgState* stt) {
  __shared__ double sh[kNT / 64];
  constexpr int RPB = kNT / TPR;
  const int lane = threadIdx.x % TPR;
  double bbp = 0.0, rrp = 0.0;
  for (int i = blockIdx.x * RPB + threadIdx.x / TPR; i < n; i += gridDim.x * RPB) {
    double s = 0.0;
    if (use_x0) {
      s = row_dot<TPR, 1>(rp[i] + lane, rp[i + 1], ci, v, x);
      s = gsum<TPR>(s);
    }
    if (lane == 0) {
      if (!use_x0) x[i] = 0.0;
      const double bi = b[i];
      const double ri = bi - s;
      r[i] = ri;
      bbp += bi * bi;
      rrp += ri * ri;
    }
  }
  // two sums: reuse the reduction twice (slots 3 and 4)
  double pb = block_sum(bbp, sh);
  double tb;
  const bool lastb = arrive(pb, partials, &stt->cnt[3], sh, &tb);
  __syncthreads();
  double pr = block_sum(rrp, sh);
  double tr;
  const bool lastr = arrive(pr, partials + gridDim.x, &stt->cnt[4], sh, &tr);
  // The workgroup that is last for the second sum has seen every first partial
  // (each workgroup arrives at the first counter before the second), so it also
  // recomputes the first total in the same fixed order.
  if (lastr) {
    double s = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) s += __builtin_nontemporal_load(partials + i);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
      tb = s;
      stt->bb = tb;
      stt->rr = tr;
      stt->iters = 0;
      stt->beta = 0.0;
      if (tb == 0.0) {
        stt->done = DONE_ZERO_RHS;
        stt->relres = 0.0;
      } else {
        const double rel = sqrt(tr) / sqrt(tb);
        stt->relres = rel;
        if (!isfinite(rel)) stt->done = DONE_BREAKDOWN;
        else if (rel <= stt->tol) stt->done = DONE_CONVERGED;
        else if (stt->maxit <= 0) stt->done = DONE_MAXIT;
      }
    }
  }
  (void)lastb;
}

template <typename FT, typename ET>
__global__ __launch_bounds__(kNT) void dense_matvec_kernel(int n, const double* __restrict__ inv,
                                                           const FT* __restrict__ f, ET* __restrict__ e,
                                                           const int* __restrict__ done) {
  if (done && *done) return;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (kNT / 64) + (threadIdx.x >> 6);
  if (row >= n) return;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += inv[(long)row * n + j] * (double)f[j];
  s = gsum<64>(s);
  if (lane == 0) e[row] = (ET)s;
}

template <typename AT, typename BT, typename YT>
__global__ __launch_bounds__(kNT) void vec_kernel(int op, int n, const AT* __restrict__ a, const BT* __restrict__ b,
                                                  YT* __restrict__ y, const int* __restrict__ done) {
  if (done && *done) return;
  for (int i = blockIdx.x * kNT + threadIdx.x; i < n; i += gridDim.x * kNT) {
    switch (op) {
      case 0: y[i] = (YT)((double)a[i] + (double)b[i]); break;
      case 1: y[i] = (YT)((double)y[i] + (double)a[i]); break;
      case 2: y[i] = (YT)(double)a[i]; break;
      default: y[i] = (YT)0; break;
    }
  }
}

__global__ __launch_bounds__(kNT) void neg_outer_kernel(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                        const double* __restrict__ lam, const double* __restrict__ x,
                                                        double* __restrict__ g) {
  constexpr int TPR = 8, RPB = kNT / TPR;
  const int lane = threadIdx.x % TPR;
  for (int i = blockIdx.x * RPB + threadIdx.x / TPR; i < n; i += gridDim.x * RPB) {
    const double li = lam[i];
    for (int k = rp[i] + lane; k < rp[i + 1]; k += TPR) g[k] = -li * x[ci[k]];
  }
}

__global__ __launch_bounds__(kNT) void to_f32_kernel(long n, const double* __restrict__ a, float* __restrict__ y) {
  for (long i = (long)blockIdx.x * kNT + threadIdx.x; i < n; i += (long)gridDim.x * kNT) y[i] = (float)a[i];
}

int grid_for(long work, int per_block, int cap = 8192) {
  long g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

// ---------------------------------------------------------------------------- launchers
#define CPC_TPR_DISPATCH(tpr, CALL) \
  switch (tpr) {                    \
    case 1: CALL(1); break;         \
    case 2: CALL(2); break;         \
    case 4: CALL(4); break;         \
    case 8: CALL(8); break;         \
    case 16: CALL(16); break;       \
    case 32: CALL(32); break;       \
    default: CALL(64); break;       \
  }

// Launches of more rows than this have waves enough to hide the dependent loads of a
// row product; smaller ones (coarse levels, the blocks of the block substitution) take
// the matrix's batched steps.
constexpr int kLatencyRows = 32768;

template <int U, typename VT, typename XT, typename FT, typename YT>
static void spmv_typed_u(hipStream_t s, const MatDev& A, int mode, const void* x, const void* f, void* y, int tpr,
                         const int* done) {
  const int rpb = kNT / tpr;
  const int grid = grid_for(A.n, rpb);
#define CPC_SPMV_CALL(T)                                                                                  \
  spmv_kernel<T, U, VT, XT, FT, YT><<<grid, kNT, 0, s>>>(A.n, A.rp, A.ci, (const VT*)A.v, (const XT*)x,  \
                                                         (const FT*)f, (YT*)y, mode, A.rid, A.mask, done)
  CPC_TPR_DISPATCH(tpr, CPC_SPMV_CALL)
#undef CPC_SPMV_CALL
}

template <typename VT, typename XT, typename FT, typename YT>
static void spmv_typed(hipStream_t s, const MatDev& A, int mode, const void* x, const void* f, void* y, int tpr,
                       const int* done) {
  const int u = A.n > kLatencyRows ? 1 : A.steps;
  if (u >= 4) spmv_typed_u<4, VT, XT, FT, YT>(s, A, mode, x, f, y, tpr, done);
  else if (u == 2) spmv_typed_u<2, VT, XT, FT, YT>(s, A, mode, x, f, y, tpr, done);
  else spmv_typed_u<1, VT, XT, FT, YT>(s, A, mode, x, f, y, tpr, done);
}

bool launch_spmv(hipStream_t s, const MatDev& A, int mode, const void* x, bool xf32, const void* f, bool ff32,
                 void* y, bool yf32, int tpr, const int* done) {
  if (A.n <= 0) return true;
  // the precision combinations the solver uses
  if (!A.fp32 && !xf32 && !ff32 && !yf32) spmv_typed<double, double, double, double>(s, A, mode, x, f, y, tpr, done);
  else if (A.fp32 && xf32 && ff32 && yf32) spmv_typed<float, float, float, float>(s, A, mode, x, f, y, tpr, done);
  else if (!A.fp32 && xf32 && !ff32 && yf32) spmv_typed<double, float, double, float>(s, A, mode, x, f, y, tpr, done);
  else return false;
  return true;
}

void launch_spmv_pq(hipStream_t s, const MatDev& A, const double* p, double* q, double* partials, PcgState* stt,
                    int tpr) {
  const int rpb = kNT / tpr;
  // at most kRedGrid workgroups: each one's arrival is a fence and an atomic on one
  // counter, which serialise (4096 workgroups took twice as long on the finest level)
  const int grid = grid_for(A.n, rpb, kRedGrid);
#define CPC_PQ_CALL(T) \
  spmv_pq_kernel<T><<<grid, kNT, 0, s>>>(A.n, A.rp, A.ci, (const double*)A.v, p, q, partials, stt)
  CPC_TPR_DISPATCH(tpr, CPC_PQ_CALL)
#undef CPC_PQ_CALL
}

void launch_update_xr(hipStream_t s, int n, double* x, double* r, const double* p, const double* q,
                      double* partials, PcgState* stt) {
  update_xr_kernel<<<grid_for(n, kNT, kRedGrid), kNT, 0, s>>>(n, x, r, p, q, partials, stt);
}

void launch_dot_rz(hipStream_t s, int n, const double* r, const double* z, double* p, double* partials,
                   PcgState* stt, bool first) {
  dot_rz_kernel<<<grid_for(n, kNT, kRedGrid), kNT, 0, s>>>(n, r, z, p, partials, stt, first ? 1 : 0);
}

void launch_update_p(hipStream_t s, int n, const double* z, double* p, PcgState* stt) {
  update_p_kernel<<<grid_for(n, kNT), kNT, 0, s>>>(n, z, p, stt);
}

void launch_pcg_init(hipStream_t s, const MatDev& A, const double* b, double* x, double* r, int use_x0,
                     double* partials, PcgState* stt, int tpr) {
  const int rpb = kNT / tpr;
  const int grid = grid_for(A.n, rpb, kRedGrid);
#define CPC_INIT_CALL(T) \
  pcg_init_kernel<T><<<grid, kNT, 0, s>>>(A.n, A.rp, A.ci, (const double*)A.v, b, x, r, use_x0, partials, stt)
  CPC_TPR_DISPATCH(tpr, CPC_INIT_CALL)
#undef CPC_INIT_CALL
}

void launch_dense_matvec(hipStream_t s, int n, const double* inv, const void* f, bool ff32, void* e, bool ef32,
                         const int* done) {
  const int grid = (n + (kNT / 64) - 1) / (kNT / 64);
  if (!ff32 && !ef32) dense_matvec_kernel<double, double><<<grid, kNT, 0, s>>>(n, inv, (const double*)f, (double*)e, done);
  else if (ff32 && ef32) dense_matvec_kernel<float, float><<<grid, kNT, 0, s>>>(n, inv, (const float*)f, (float*)e, done);
  else if (ff32) dense_matvec_kernel<float, double><<<grid, kNT, 0, s>>>(n, inv, (const float*)f, (double*)e, done);
  else dense_matvec_kernel<double, float><<<grid, kNT, 0, s>>>(n, inv, (const double*)f, (float*)e, done);
}

void launch_vec(hipStream_t s, int op, int n, const void* a, bool af32, const void* b, bool bf32, void* y, bool yf32,
                const int* done) {
  if (n <= 0) return;
  const int grid = grid_for(n, kNT);
#define CPC_VEC(A_, B_, Y_) \
  vec_kernel<A_, B_, Y_><<<grid, kNT, 0, s>>>(op, n, (const A_*)a, (const B_*)b, (Y_*)y, done)
  const int key = (af32 ? 4 : 0) | (bf32 ? 2 : 0) | (yf32 ? 1 : 0);
  switch (key) {
    case 0: CPC_VEC(double, double, double); break;
    case 1: CPC_VEC(double, double, float); break;
    case 2: CPC_VEC(double, float, double); break;
    case 3: CPC_VEC(double, float, float); break;
    case 4: CPC_VEC(float, double, double); break;
    case 5: CPC_VEC(float, double, float); break;
    case 6: CPC_VEC(float, float, double); break;
    default: CPC_VEC(float, float, float); break;
  }
#undef CPC_VEC
}

void launch_neg_outer(hipStream_t s, const MatDev& A, const double* lam, const double* x, double* g) {
  neg_outer_kernel<<<grid_for(A.n, kNT / 8), kNT, 0, s>>>(A.n, A.rp, A.ci, lam, x, g);
}

void launch_to_f32(hipStream_t s, int64_t n, const double* a, float* y) {
  to_f32_kernel<<<grid_for(n, kNT), kNT, 0, s>>>((long)n, a, y);
}

}  // namespace cpc
