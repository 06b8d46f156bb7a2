// Two-point-flux pressure matrix of the model problem of Section 4 (c = 0) on an
// nx x ny x nz grid of unit cells, and the chain rule of a misfit gradient through
// it (the differentiable form of the solve).
//
// Matrix: a_ij = -T_ij for face neighbours, a_ii = sum of the cell's T plus
// T_b = 2 k_i on each Dirichlet x-face; T = 2 s k_a k_b / (k_a + k_b) with s = 1 on
// x/y faces and s = kz_ratio on z faces; k = exp(log k). Entries of row c are stored
// in column order: z-, y-, x-, diagonal, x+, y+, z+ (those that exist).
//
// Gradient: with lam = A^{-1} (dL/dx) and dL/da_ij = -lam_i x_j, a face f = (a, b)
// contributes dL/dT_f = -(lam_a - lam_b)(x_a - x_b) and dT_f/dlog k_a =
// 2 s k_a k_b^2 / (k_a + k_b)^2; a Dirichlet face of cell c contributes
// -T_b lam_c x_c (dT_b/dlog k_c = T_b).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cpc {

namespace {

__device__ __forceinline__ double face_t(double ka, double kb, double s) {
  const double a = s * ka, b = s * kb;
  return 2.0 * a * b / (a + b);
}

__device__ __forceinline__ double face_dt(double ka, double kb, double s) {  // dT/dlog k_a
  const double a = s * ka, b = s * kb;
  const double d = a + b;
  return 2.0 * a * b * b / (d * d);
}

__global__ __launch_bounds__(256) void tpfa_values_kernel(int nx, int ny, int nz, double kz, int dirichlet,
                                                          const double* __restrict__ logk,
                                                          const int* __restrict__ rp, double* __restrict__ val) {
  const long N = (long)nx * ny * nz;
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
    const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((long)nx * ny));
    const double kc = exp(logk[c]);
    const long nxy = (long)nx * ny;
    double t[6] = {0, 0, 0, 0, 0, 0};
    const bool has[6] = {k > 0, j > 0, i > 0, i < nx - 1, j < ny - 1, k < nz - 1};
    const long off[6] = {-nxy, -nx, -1, 1, nx, nxy};
    const double sc[6] = {kz, 1.0, 1.0, 1.0, 1.0, kz};
    double diag = 0.0;
    for (int f = 0; f < 6; ++f)
      if (has[f]) {
        t[f] = face_t(kc, exp(logk[c + off[f]]), sc[f]);
        diag += t[f];
      }
    if (dirichlet) {
      if (i == 0) diag += 2.0 * kc;
      if (i == nx - 1) diag += 2.0 * kc;
    }
    int p = rp[c];
    for (int f = 0; f < 3; ++f)
      if (has[f]) val[p++] = -t[f];
    val[p++] = diag;
    for (int f = 3; f < 6; ++f)
      if (has[f]) val[p++] = -t[f];
  }
}

__global__ __launch_bounds__(256) void tpfa_grad_kernel(int nx, int ny, int nz, double kz, int dirichlet,
                                                        const double* __restrict__ logk,
                                                        const double* __restrict__ lam, const double* __restrict__ x,
                                                        double* __restrict__ g) {
  const long N = (long)nx * ny * nz;
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
    const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((long)nx * ny));
    const double kc = exp(logk[c]);
    const long nxy = (long)nx * ny;
    const bool has[6] = {k > 0, j > 0, i > 0, i < nx - 1, j < ny - 1, k < nz - 1};
    const long off[6] = {-nxy, -nx, -1, 1, nx, nxy};
    const double sc[6] = {kz, 1.0, 1.0, 1.0, 1.0, kz};
    const double lc = lam[c], xc = x[c];
    double acc = 0.0;
    for (int f = 0; f < 6; ++f)
      if (has[f]) {
        const long nb = c + off[f];
        const double dldt = -(lc - lam[nb]) * (xc - x[nb]);
        acc += face_dt(kc, exp(logk[nb]), sc[f]) * dldt;
      }
    if (dirichlet) {
      if (i == 0) acc += -(2.0 * kc) * lc * xc;
      if (i == nx - 1) acc += -(2.0 * kc) * lc * xc;
    }
    g[c] = acc;
  }
}

int tgrid(long n) {
  long g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

void launch_tpfa_values(hipStream_t s, int nx, int ny, int nz, double kz, int dirichlet, const double* logk,
                        const int* rp, double* val) {
  tpfa_values_kernel<<<tgrid((long)nx * ny * nz), 256, 0, s>>>(nx, ny, nz, kz, dirichlet, logk, rp, val);
}

void launch_tpfa_grad(hipStream_t s, int nx, int ny, int nz, double kz, int dirichlet, const double* logk,
                      const double* lam, const double* x, double* g) {
  tpfa_grad_kernel<<<tgrid((long)nx * ny * nz), 256, 0, s>>>(nx, ny, nz, kz, dirichlet, logk, lam, x, g);
}

}  // namespace cpc
