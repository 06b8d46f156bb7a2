// One lane's part of a CSR row product (device code of the HIP sources).
#pragma once
#include <hip/hip_runtime.h>

namespace cpc {

// Entries p, p + TPR, ... < e of a row (columns ci, values v) times x, added in that
// order. U of them are taken at once: their columns and values are loaded, then the U
// x entries, then the products added, so a row of up to U TPR entries costs two
// dependent memory rounds instead of two per TPR entries; that pays where a launch is
// too small to hide the rounds behind other waves. A step past the row reads the lane's
// first entry again and its product is not added (U = 1 is the plain loop).
template <int TPR, int U, typename VT, typename XT>
__device__ __forceinline__ double row_dot(int p, int e, const int* __restrict__ ci, const VT* __restrict__ v,
                                          const XT* __restrict__ x) {
  double s = 0.0;
  for (; p < e; p += U * TPR) {
    int c[U];
    VT w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = p + u * TPR < e ? p + u * TPR : p;
      c[u] = ci[q];
      w[u] = v[q];
    }
    double xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = (double)x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (p + u * TPR < e) s += (double)w[u] * xv[u];
  }
  return s;
}

}  // namespace cpc
