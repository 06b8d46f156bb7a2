// FP64 matrix products on the matrix cores for the setup of the explicit inverses.
//
// The span merges of the triangular inverse (dense_tri.hip) are two dense products
// per pair of adjacent inverted spans; all pairs of one span length are independent,
// so one launch takes every pair (the batch index picks the pair's operands at fixed
// element strides). Each workgroup (four waves) computes a 64 x 64 tile of the output
// from 64 x 16 and 16 x 64 tiles of the operands staged in LDS; each wave holds a
// 32 x 32 sub-tile as four 16 x 16 accumulators of v_mfma_f64_16x16x4f64
// (A operand: lane l holds row l % 16, inner index l / 16; B operand: column l % 16,
// inner index l / 16; result: register r of lane l holds row l / 16 + 4 r of column
// l % 16, as measured on gfx950).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cpc {

namespace {

constexpr int kGT = 64;  // output tile edge
constexpr int kGK = 16;  // inner step staged per round

typedef double dvec4 __attribute__((ext_vector_type(4)));

// O[z] = alpha * L[z] R[z] for z = blockIdx.z: L[z] rows x inner (row stride ldl),
// R[z] inner x cols (ldr), O[z] rows x cols (ldo), row-major; entry z's operands start
// z * sl, z * sr, z * so elements after the first ones; the last entry has rows_last
// rows and inner_last inner indices (a shorter last span).
__global__ __launch_bounds__(256) void dgemm_mfma_kernel(const double* __restrict__ L, long sl, int ldl,
                                                         const double* __restrict__ R, long sr, int ldr,
                                                         double* __restrict__ O, long so, int ldo, int rows,
                                                         int rows_last, int inner, int inner_last, int cols, int nb,
                                                         double alpha) {
  __shared__ double Ls[kGT][kGK + 1];
  __shared__ double Rs[kGK][kGT + 1];
  const int z = blockIdx.z;
  const int M = z == nb - 1 ? rows_last : rows;
  const int K = z == nb - 1 ? inner_last : inner;
  const int N = cols;
  const int r0 = blockIdx.y * kGT, c0 = blockIdx.x * kGT;
  if (r0 >= M || c0 >= N) return;  // the whole workgroup: a tile past a shorter last entry
  L += z * sl;
  R += z * sr;
  O += z * so;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  dvec4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = dvec4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += kGK) {
#pragma unroll
    for (int e = tid; e < kGT * kGK; e += 256) {
      const int i = e / kGK, k = e % kGK;
      const int gi = r0 + i, gk = k0 + k;
      Ls[i][k] = (gi < M && gk < K) ? L[(long)gi * ldl + gk] : 0.0;
    }
#pragma unroll
    for (int e = tid; e < kGK * kGT; e += 256) {
      const int k = e / kGT, j = e % kGT;
      const int gk = k0 + k, gj = c0 + j;
      Rs[k][j] = (gk < K && gj < N) ? R[(long)gk * ldr + gj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const double a = Ls[wr + bi * 16 + li][kk + lk];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          const double b = Rs[kk + lk][wc + bj * 16 + li];
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[bi][bj], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wr + bi * 16 + lk + 4 * r, col = c0 + wc + bj * 16 + li;
        if (row < M && col < N) O[(long)row * ldo + col] = alpha * acc[bi][bj][r];
      }
}

}  // namespace

bool launch_dgemm_batched(hipStream_t s, const double* L, long sl, int ldl, const double* R, long sr, int ldr,
                          double* O, long so, int ldo, int rows, int rows_last, int inner, int inner_last, int cols,
                          int nb, double alpha) {
  if (nb <= 0 || rows <= 0 || cols <= 0 || inner <= 0 || rows_last <= 0 || rows_last > rows || inner_last <= 0 ||
      inner_last > inner || nb > 65535)
    return false;
  const dim3 grid((cols + kGT - 1) / kGT, (rows + kGT - 1) / kGT, nb);
  dgemm_mfma_kernel<<<grid, 256, 0, s>>>(L, sl, ldl, R, sr, ldr, O, so, ldo, rows, rows_last, inner, inner_last,
                                         cols, nb, alpha);
  return hipGetLastError() == hipSuccess;
}

}  // namespace cpc
