// Batched PCG for many independent systems of different sizes, solved together.
//
// The systems' vectors are concatenated. Rows are cut into chunks that never
// straddle two systems; one workgroup handles one chunk. Every system has its own
// scalars (rho, <p,q>, alpha, beta, ||r||, ||b||, iteration count, stop flag): each
// reduction writes one partial per chunk, and the last chunk of a system to arrive
// sums that system's partials in chunk order (deterministic) and updates its
// scalars. A system that has stopped skips all of its chunks, so its iterate and
// iteration count stay exact while the others continue.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "csr_row.hpp"
#include "wave_sum.hpp"

namespace cpc {

namespace {

constexpr int kNT = 256;

__device__ double bsum(double v, double* sh) {
  v = gsum<64>(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  return s;
}

// chunk c publishes its partial; true (all threads) in the last chunk of system s,
// whose thread 0 then holds the system total in *total.
__device__ bool sys_arrive(double part, const BatchDev& bd, int slot, int c, int s, double* sh, double* total) {
  __shared__ int s_last;
  double* partials = bd.partials + (size_t)slot * bd.nchunks;
  unsigned* cnt = bd.cnt + (size_t)slot * bd.nsys;
  const int c0 = bd.sys_chunk[s], c1 = bd.sys_chunk[s + 1];
  if (threadIdx.x == 0) {
    partials[c] = part;
    __threadfence();
    const unsigned t = atomicAdd(cnt + s, 1u);
    s_last = (t == (unsigned)(c1 - c0 - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  double acc = 0.0;
  for (int k = c0 + threadIdx.x; k < c1; k += blockDim.x) acc += __builtin_nontemporal_load(partials + k);
  acc = bsum(acc, sh);
  if (threadIdx.x == 0) {
    *total = acc;
    cnt[s] = 0u;
  }
  return true;
}

template <int TPR>
__global__ __launch_bounds__(kNT) void bspmv_pq_kernel(BatchDev bd, const int* __restrict__ rp,
                                                       const int* __restrict__ ci, const double* __restrict__ v,
                                                       const double* __restrict__ p, double* __restrict__ q) {
  __shared__ double sh[kNT / 64];
  const int c = blockIdx.x;
  const int s = bd.chunk_sys[c];
  if (bd.done[s]) return;
  const int r0 = bd.chunk_row[c], r1 = bd.chunk_row[c + 1];
  const int lane = threadIdx.x % TPR;
  double acc = 0.0;
  for (int i = r0 + threadIdx.x / TPR; i < r1; i += kNT / TPR) {
    double t = row_dot<TPR, 1>(rp[i] + lane, rp[i + 1], ci, v, p);
    t = gsum<TPR>(t);
    if (lane == 0) {
      q[i] = t;
      acc += t * p[i];
    }
  }
  double part = bsum(acc, sh), tot;
  if (sys_arrive(part, bd, 0, c, s, sh, &tot) && threadIdx.x == 0) {
    bd.pq[s] = tot;
    if (!(tot > 0.0) || !isfinite(tot)) bd.done[s] = DONE_BREAKDOWN;
    else bd.alpha[s] = bd.rz[s] / tot;
  }
}

__global__ __launch_bounds__(kNT) void bupdate_xr_kernel(BatchDev bd, double* __restrict__ x, double* __restrict__ r,
                                                         const double* __restrict__ p, const double* __restrict__ q) {
  __shared__ double sh[kNT / 64];
  const int c = blockIdx.x;
  const int s = bd.chunk_sys[c];
  if (bd.done[s]) return;
  const int r0 = bd.chunk_row[c], r1 = bd.chunk_row[c + 1];
  const double a = bd.alpha[s];
  double acc = 0.0;
  for (int i = r0 + threadIdx.x; i < r1; i += kNT) {
    x[i] = x[i] + a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  double part = bsum(acc, sh), tot;
  if (sys_arrive(part, bd, 1, c, s, sh, &tot) && threadIdx.x == 0) {
    bd.rr[s] = tot;
    const int it = bd.iters[s] + 1;
    bd.iters[s] = it;
    const double rel = sqrt(tot) / sqrt(bd.bb[s]);
    bd.relres[s] = rel;
    if (!isfinite(rel)) bd.done[s] = DONE_BREAKDOWN;
    else if (rel <= (*bd.tol_dev)) bd.done[s] = DONE_CONVERGED;
    else if (it >= (*bd.maxit_dev)) bd.done[s] = DONE_MAXIT;
  }
}

__global__ __launch_bounds__(kNT) void bdot_rz_kernel(BatchDev bd, const double* __restrict__ r,
                                                      const double* __restrict__ z, double* __restrict__ p,
                                                      int first) {
  __shared__ double sh[kNT / 64];
  const int c = blockIdx.x;
  const int s = bd.chunk_sys[c];
  if (bd.done[s]) return;
  const int r0 = bd.chunk_row[c], r1 = bd.chunk_row[c + 1];
  double acc = 0.0;
  for (int i = r0 + threadIdx.x; i < r1; i += kNT) {
    const double zi = z[i];
    acc += r[i] * zi;
    if (first) p[i] = zi;
  }
  double part = bsum(acc, sh), tot;
  if (sys_arrive(part, bd, 2, c, s, sh, &tot) && threadIdx.x == 0) {
    if (!(tot > 0.0) || !isfinite(tot)) {
      bd.done[s] = DONE_BREAKDOWN;
    } else {
      if (!first) bd.beta[s] = tot / bd.rz[s];
      bd.rz[s] = tot;
    }
  }
}

__global__ __launch_bounds__(kNT) void bupdate_p_kernel(BatchDev bd, const double* __restrict__ z,
                                                        double* __restrict__ p) {
  const int c = blockIdx.x;
  const int s = bd.chunk_sys[c];
  if (bd.done[s]) return;
  const int r0 = bd.chunk_row[c], r1 = bd.chunk_row[c + 1];
  const double be = bd.beta[s];
  for (int i = r0 + threadIdx.x; i < r1; i += kNT) p[i] = z[i] + be * p[i];
}

// r = b, x = 0; ||b||^2 per system; relres test before the first iteration.
__global__ __launch_bounds__(kNT) void binit_kernel(BatchDev bd, const double* __restrict__ b, double* __restrict__ x,
                                                    double* __restrict__ r) {
  __shared__ double sh[kNT / 64];
  const int c = blockIdx.x;
  const int s = bd.chunk_sys[c];
  const int r0 = bd.chunk_row[c], r1 = bd.chunk_row[c + 1];
  double acc = 0.0;
  for (int i = r0 + threadIdx.x; i < r1; i += kNT) {
    const double bi = b[i];
    x[i] = 0.0;
    r[i] = bi;
    acc += bi * bi;
  }
  double part = bsum(acc, sh), tot;
  if (sys_arrive(part, bd, 3, c, s, sh, &tot) && threadIdx.x == 0) {
    bd.bb[s] = tot;
    bd.rr[s] = tot;
    bd.iters[s] = 0;
    bd.beta[s] = 0.0;
    if (tot == 0.0) {
      bd.done[s] = DONE_ZERO_RHS;
      bd.relres[s] = 0.0;
    } else {
      bd.relres[s] = 1.0;
      bd.done[s] = (1.0 <= (*bd.tol_dev)) ? DONE_CONVERGED : ((*bd.maxit_dev) <= 0 ? DONE_MAXIT : DONE_RUNNING);
    }
  }
}

// Coarsest levels of several systems: e = inv_s f on each system's segment.
__global__ __launch_bounds__(kNT) void bdense_kernel(DenseListDev dl, const void* f, void* e, int fp32,
                                                     const int* __restrict__ done) {
  if (done && *done) return;
  const int blk = blockIdx.x;
  const int ent = dl.blk_entry[blk];
  if (masked(dl.mask, ent)) return;  // a system that has stopped
  const int n0 = dl.n[ent];
  const int off = dl.off[ent];
  const double* inv = dl.inv + dl.inv_off[ent];
  const int row = dl.blk_row0[blk] + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n0) return;
  double s = 0.0;
  if (fp32) {
    const float* ff = reinterpret_cast<const float*>(f) + off;
    for (int j = lane; j < n0; j += 64) s += inv[(long)row * n0 + j] * (double)ff[j];
  } else {
    const double* ff = reinterpret_cast<const double*>(f) + off;
    for (int j = lane; j < n0; j += 64) s += inv[(long)row * n0 + j] * ff[j];
  }
  s = gsum<64>(s);
  if (lane == 0) {
    if (fp32) reinterpret_cast<float*>(e)[off + row] = (float)s;
    else reinterpret_cast<double*>(e)[off + row] = s;
  }
}

}  // namespace

#define CPC_TPR_SWITCH(tpr, CALL) \
  switch (tpr) {                  \
    case 1: CALL(1); break;       \
    case 2: CALL(2); break;       \
    case 4: CALL(4); break;       \
    case 8: CALL(8); break;       \
    case 16: CALL(16); break;     \
    case 32: CALL(32); break;     \
    default: CALL(64); break;     \
  }

void launch_bspmv_pq(hipStream_t s, const BatchDev& bd, const MatDev& A, const double* p, double* q, int tpr) {
#define CPC_B(T) bspmv_pq_kernel<T><<<bd.nchunks, kNT, 0, s>>>(bd, A.rp, A.ci, (const double*)A.v, p, q)
  CPC_TPR_SWITCH(tpr, CPC_B)
#undef CPC_B
}

void launch_bupdate_xr(hipStream_t s, const BatchDev& bd, double* x, double* r, const double* p, const double* q) {
  bupdate_xr_kernel<<<bd.nchunks, kNT, 0, s>>>(bd, x, r, p, q);
}

void launch_bdot_rz(hipStream_t s, const BatchDev& bd, const double* r, const double* z, double* p, bool first) {
  bdot_rz_kernel<<<bd.nchunks, kNT, 0, s>>>(bd, r, z, p, first ? 1 : 0);
}

void launch_bupdate_p(hipStream_t s, const BatchDev& bd, const double* z, double* p) {
  bupdate_p_kernel<<<bd.nchunks, kNT, 0, s>>>(bd, z, p);
}

void launch_binit(hipStream_t s, const BatchDev& bd, const double* b, double* x, double* r) {
  binit_kernel<<<bd.nchunks, kNT, 0, s>>>(bd, b, x, r);
}

void launch_bdense(hipStream_t s, const DenseListDev& dl, const void* f, void* e, bool fp32, const int* done) {
  if (dl.nblk <= 0) return;
  bdense_kernel<<<dl.nblk, kNT, 0, s>>>(dl, f, e, fp32 ? 1 : 0, done);
}

}  // namespace cpc
