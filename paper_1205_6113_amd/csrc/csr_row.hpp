// One lane's part of a CSR row product (device code of the HIP sources).
#pragma once
#include <hip/hip_runtime.h>

namespace cpc {

// Entries p, p + TPR, ... < e of a row (columns ci, values v) times x, added in that
// order. Four of them are taken at once: their columns and values are loaded, then the
// four x entries, then the products added, so a row of up to 4 TPR entries costs two
// dependent memory rounds instead of two per TPR entries. A step past the row reads the
// lane's first entry again and its product is not added.
template <int TPR, typename VT, typename XT>
__device__ __forceinline__ double row_dot(int p, int e, const int* __restrict__ ci, const VT* __restrict__ v,
                                          const XT* __restrict__ x) {
  constexpr int U = 4;
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
