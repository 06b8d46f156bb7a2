// Dense explicit inverses of the Gauss-Seidel factor T = D + L on small levels.
//
// On the coarse levels of a classical AMG hierarchy the forward sweep T^{-1} f has a
// dependency depth close to the number of rows divided by a handful, so a
// level-scheduled sweep there is bound by the latency of thousands of dependent steps
// rather than by memory traffic. With hundreds of gigabytes of HBM the inverse of T
// can be held explicitly instead: the forward sweep becomes the lower-triangular
// matrix-vector product y = T^{-1} f, and since D + U = T^T for symmetric A the
// backward sweep (D+U)^{-1} g becomes the transposed product y = T^{-T} g. Both read
// the n(n+1)/2 stored entries once and are bound by HBM bandwidth.
//
// Setup (per system of a level, n rows): T is scattered into a zeroed dense n x n
// row-major array; the 128 x 128 diagonal blocks are inverted in place by
// substitution in LDS; then, for spans of 128, 256, 512, ... rows, each pair of
// adjacent inverted spans [a, a+s) and [a+s, b) gets its off-diagonal block
// B <- -C^{-1} B A^{-1} from two matrix products (FP64 on the matrix cores,
// dense_gemm.hip), where A^{-1}, C^{-1} are the inverted diagonal spans. The result is
// T^{-1}, lower triangular.
//
// Products: y = T^{-1} f by one workgroup per eight rows, four from each end of the
// system (coalesced row reads, the vector from L2). y = T^{-T} g: on smaller systems from a stored transpose, row by row like the
// forward product; on larger ones by items (column block of 512, chunk of 1024 rows)
// whose partial column sums go to a buffer and are added in chunk order
// (deterministic), which reads each stored entry once without a second copy.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "kernels.hpp"
#include "wave_sum.hpp"

namespace cpc {

namespace {

constexpr int kLeaf = 128;  // diagonal blocks inverted by substitution
constexpr int kNT = 256;

// The diagonal block of T on rows and columns [voff, voff + n) of a CSR into the dense
// row-major array M (leading dimension n): lower triangle only (upper entries stay zero).
__global__ __launch_bounds__(kNT) void scatter_lower_kernel(int n, int voff, const int* __restrict__ rp,
                                                           const int* __restrict__ ci,
                                                           const double* __restrict__ v, double* __restrict__ M) {
  const long ld = dense_ld(n);
  for (int i = blockIdx.x * kNT + threadIdx.x; i < n; i += gridDim.x * kNT) {
    const int r = voff + i;
    for (int p = rp[r]; p < rp[r + 1]; ++p) {
      const int j = ci[p] - voff;
      if (j >= 0 && j <= i) M[i * ld + j] = v[p];  // the diagonal block only
    }
  }
}

// In-place inverse of the lower-triangular diagonal block of M starting at row and
// column b * kLeaf (size nb <= kLeaf). Row by row: x_ii = 1 / t_ii and, for j < i,
// x_ij = -(sum_{k=j}^{i-1} t_ik x_kj) / t_ii, with the finished rows of X in LDS.
__global__ __launch_bounds__(kLeaf) void leaf_inverse_kernel(int n, double* __restrict__ M) {
  __shared__ double X[kLeaf][kLeaf + 1];
  __shared__ double trow[kLeaf];
  const int b0 = blockIdx.x * kLeaf;
  const int nb = min(kLeaf, n - b0);
  const long ld = dense_ld(n);
  const int j = threadIdx.x;
  for (int i = 0; i < nb; ++i) {
    if (j < nb) trow[j] = M[(b0 + i) * ld + b0 + j];
    __syncthreads();
    const double dinv = 1.0 / trow[i];
    double x = 0.0;
    if (j < i) {
      double s0 = 0.0, s1 = 0.0;
      int k = j;
      for (; k + 1 < i; k += 2) {
        s0 += trow[k] * X[k][j];
        s1 += trow[k + 1] * X[k + 1][j];
      }
      if (k < i) s0 += trow[k] * X[k][j];
      x = -(s0 + s1) * dinv;
    } else if (j == i) {
      x = dinv;
    }
    if (j < nb) X[i][j] = x;
    __syncthreads();
  }
  for (int i = 0; i < nb; ++i)
    if (j < nb) M[(b0 + i) * ld + b0 + j] = X[i][j];
}

// Y = X^T for an n x n row-major X (row stride dense_ld(n)), 32 x 32 tiles through LDS.
template <typename MT>
__global__ __launch_bounds__(kNT) void transpose_kernel(int n, const MT* __restrict__ X, MT* __restrict__ Y) {
  __shared__ MT tile[32][33];
  const long ld = dense_ld(n);
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int r = ty; r < 32; r += 8) {
    const int i = by + r, j = bx + tx;
    if (i < n && j < n) tile[r][tx] = X[i * ld + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + r, j = by + tx;
    if (i < n && j < n) Y[i * ld + j] = tile[tx][r];
  }
}

template <typename MT>
__global__ __launch_bounds__(kNT) void to_type_kernel(long n, const double* __restrict__ a, MT* __restrict__ y) {
  for (long i = (long)blockIdx.x * kNT + threadIdx.x; i < n; i += (long)gridDim.x * kNT) y[i] = (MT)a[i];
}

// 16-byte vector of MT, loaded non-temporally: the inverses are streamed once per
// product, and marking them so keeps them from displacing what the small kernels between
// two products read (the off-block rows, the level vectors, the convergence flag).
template <typename MT>
struct Vec16 {
  static constexpr int N = 16 / sizeof(MT);
  using T = MT __attribute__((ext_vector_type(N)));
  __device__ static T load(const char* p) { return __builtin_nontemporal_load(reinterpret_cast<const T*>(p)); }
  __device__ static double at(const T& v, int k) { return (double)v[k]; }
};

// Entries of the flat vector list a thread loads before it uses any of them, at most: 8 x
// (4 row vectors + 2 input entries) in FP64, 4 x (4 + 4) in FP32 (a vector spans twice
// the columns), about 200 registers, two waves per SIMD. Launches over smaller systems
// take fewer steps per batch (row_steps_for), so that no thread issues loads of steps
// past its list.
template <typename MT>
constexpr int row_steps() { return sizeof(MT) == 8 ? 8 : 4; }

// One item's products into acc[0..8) (rows of group A, then of group B); the list and
// the loads are as described at the kernel below. FV: the input entries of a column
// vector are read as one 16-byte vector, which needs the system's part of the input
// 16-byte aligned and n a multiple of the vector width (every vector then lies inside
// it); otherwise they are read one by one, the index clamped to the system.
template <bool FV, typename MT, typename XT, int D>
__device__ __forceinline__ void item_products(const char* __restrict__ Mb, const char* __restrict__ fb, int n,
                                              int sa, int la, int sb, int len, const unsigned (&oa)[kHalfRows],
                                              const unsigned (&ob)[kHalfRows], double (&acc)[2 * kHalfRows]) {
  using V = Vec16<MT>;
  using VT = typename V::T;
  constexpr int W = V::N, H = kHalfRows;
  static_assert(!FV || sizeof(XT) == sizeof(MT), "vector input reads assume input and inverse of one type");
  // one step's loads: the four row vectors at list entry vd (the first entry again past
  // the list) and the input entries there; sel 1: group A, 0: group B, -1: past the list
  auto load_step = [&](int vd, int vfirst, VT (&mr)[H], XT (&fr)[W], double& sl) {
    const int v = vd < len ? vd : vfirst;
    const bool ina = v < la;
    const int c = ina ? sa + v : sb + (v - la);
    const unsigned oc = (unsigned)c * (unsigned)sizeof(VT);
#pragma unroll
    for (int r = 0; r < H; ++r) mr[r] = V::load(Mb + ((ina ? oa[r] : ob[r]) + oc));
    if constexpr (FV) {
      using FT = typename Vec16<XT>::T;
      const FT t = *reinterpret_cast<const FT*>(fb + oc);
#pragma unroll
      for (int k = 0; k < W; ++k) fr[k] = t[k];
    } else {
#pragma unroll
      for (int k = 0; k < W; ++k)
        fr[k] = *reinterpret_cast<const XT*>(fb + (unsigned)min(c * W + k, n - 1) * (unsigned)sizeof(XT));
    }
    sl = vd < len ? (ina ? 1.0 : 0.0) : -1.0;
  };
  auto use_step = [&](const VT (&mr)[H], const XT (&fr)[W], double sl) {
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const double fk = (double)fr[k];
      const double fka = sl == 1.0 ? fk : 0.0, fkb = sl == 0.0 ? fk : 0.0;
#pragma unroll
      for (int r = 0; r < H; ++r) {
        const double e = V::at(mr[r], k);
        acc[r] = fma(e, fka, acc[r]);
        acc[H + r] = fma(e, fkb, acc[H + r]);
      }
    }
  };
  for (int v0 = threadIdx.x; v0 < len; v0 += D * kNT) {
    VT m[D][H];
    XT fv[D][W];
    double sel[D];
#pragma unroll
    for (int d = 0; d < D; ++d) load_step(v0 + d * kNT, v0, m[d], fv[d], sel[d]);
    // when fewer than kNT entries would be left for another round (two per item of a
    // 4096-row block: its groups read n + 4 columns), the lanes they fall on load them
    // with this batch instead of in a dependent second round
    const int rest = len - (v0 - (int)threadIdx.x) - D * kNT;  // uniform
    const bool tail_round = rest > 0 && rest <= kNT;
    VT mt[H];
    XT ft[W];
    double st = -1.0;
    if (tail_round && v0 + D * kNT < len) load_step(v0 + D * kNT, v0, mt, ft, st);
#pragma unroll
    for (int d = 0; d < D; ++d) use_step(m[d], fv[d], sel[d]);
    if (tail_round) {
      if (v0 + D * kNT < len) use_step(mt, ft, st);
      break;
    }
  }
}

// y = M f with M lower (y = T^{-1} f) or upper (y = T^{-T} g from the stored
// transpose) triangular. An item holds two groups of at most four rows, one from each end
// of the system (rows 4k.. and the mirrored rows from the bottom), so that every item
// carries about the same number of entries and no workgroup of a launch lags far behind
// the others. Each group reads the 16-byte vectors that cover its rows' triangle: lower
// rows [a, a+4) the columns [0, a+4), upper rows the columns [a, n), rounded out to whole
// vectors. The few entries this takes beyond a row's own triangle, and the padding
// columns past n, are zeros of the stored square, so they add nothing (the input entry
// index is clamped to the system there). A group of fewer than four rows reads its last
// row again in place of the missing ones (those sums are never stored). The two groups'
// vector ranges are laid end to end and dealt to the threads as one list (thread t takes
// entries t, t + 256, ...); each entry is the four row vectors at one column vector and
// the input entries there, shared by the four rows. A thread issues the loads of
// several entries before it uses any of them, with no branch between, so most of a
// launch's traffic is in flight at once rather than in a chain of dependent rounds. An
// entry's products go to its own group's sums; the other group's sums take exact zeros
// (a product with a zero factor of finite entries). The 256 partials of each row are
// then added in a fixed order: within each wave by lane exchanges taken for all eight
// rows at once (DPP and one swizzle, so no row's chain of waits holds up the others),
// then the four waves' sums.
// At most two waves per SIMD: the compiler may then keep a whole batch of loads in
// registers (it otherwise schedules for eight waves and issues one load at a time).
template <bool UPPER, typename MT, typename XT, int D>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(1, 2))) void gemv_tri_rows_kernel(
    DenseTriDev dt, const XT* __restrict__ f, XT* __restrict__ y, const int* __restrict__ done) {
  using V = Vec16<MT>;
  using VT = typename V::T;
  constexpr int W = V::N, H = kHalfRows;
  __shared__ double red[kNT / 64][2 * H];
  if (done && *done) return;
  int n, a0, b0, na, nb, voff;
  long moff;
  if (dt.one_n > 0) {  // item k: rows 4k.. and the mirrored group m-1-k, if it lies below
    if (masked(dt.mask, dt.one_sys)) return;
    n = dt.one_n;
    voff = dt.one_voff;
    moff = dt.one_moff;
    const int m = (n + H - 1) / H, k = blockIdx.x, kb = m - 1 - k;
    a0 = k * H;
    na = min(H, n - a0);
    b0 = kb > k ? kb * H : 0;
    nb = kb > k ? min(H, n - b0) : 0;
  } else {
    const int4 iv = dt.item_n[blockIdx.x];
    const int s = iv.x;
    if (masked(dt.mask, s)) return;  // a block of a system that has stopped
    n = dt.n[s];
    a0 = iv.y;
    b0 = iv.z;
    na = iv.w & 15;
    nb = (iv.w >> 4) & 15;
    voff = dt.voff[s];
    moff = dt.moff[s];
  }
  const long vs = dense_ld(n) / W;  // row stride in vectors
  const VT* __restrict__ M = reinterpret_cast<const VT*>(reinterpret_cast<const MT*>(UPPER ? dt.MT : dt.M) + moff);
  const XT* __restrict__ fs = f + voff;
  // the groups' column-vector ranges [sa, sa + la) and [sb, sb + lb)
  const int nv = (n + W - 1) / W;
  const int sa = UPPER ? a0 / W : 0, la = UPPER ? nv - sa : (a0 + na + W - 1) / W;
  const int sb = UPPER ? b0 / W : 0, lb = nb == 0 ? 0 : (UPPER ? nv - sb : (b0 + nb + W - 1) / W);
  const int len = la + lb;
  // byte offsets from M fit 32 bits (a system's inverse is at most 16384^2 entries), so
  // each load takes the uniform base and one per-lane register
  const char* __restrict__ Mb = reinterpret_cast<const char*>(M);
  const char* __restrict__ fb = reinterpret_cast<const char*>(fs);
  unsigned oa[H], ob[H];
#pragma unroll
  for (int r = 0; r < H; ++r) {
    oa[r] = (unsigned)((a0 + min(r, na - 1)) * vs) * (unsigned)sizeof(VT);
    ob[r] = (unsigned)((b0 + min(r, max(nb - 1, 0))) * vs) * (unsigned)sizeof(VT);
  }
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double acc[2 * H];
#pragma unroll
  for (int r = 0; r < 2 * H; ++r) acc[r] = 0.0;
  if ((reinterpret_cast<unsigned long>(fs) & 15) == 0 && n % W == 0)
    item_products<true, MT, XT, D>(Mb, fb, n, sa, la, sb, len, oa, ob, acc);
  else
    item_products<false, MT, XT, D>(Mb, fb, n, sa, la, sb, len, oa, ob, acc);
  wave_sums(acc);  // valid in lane 0
  if (lane == 0)
#pragma unroll
    for (int r = 0; r < 2 * H; ++r) red[w][r] = acc[r];
  __syncthreads();
  if (tid < 2 * H) {
    const bool ok = tid < H ? tid < na : tid - H < nb;
    const int row = tid < H ? a0 + tid : b0 + tid - H;
    if (ok) y[voff + row] = (XT)((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]));
  }
}

// Partial column sums of T^{-T} g: item (system, first column c0, first row r0, slot);
// each thread owns columns c0 + 2t, c0 + 2t + 1 and adds rows [max(r0, c0), r0 + chunk).
template <typename MT, typename XT>
__global__ __launch_bounds__(kNT) void gemv_lower_t_part_kernel(DenseTriDev dt, const XT* __restrict__ g,
                                                                const int* __restrict__ done) {
  if (done && *done) return;
  const int4 it = dt.item_t[blockIdx.x];
  const int s = it.x;
  const int n = dt.n[s];
  const int voff = dt.voff[s];
  const MT* __restrict__ M = reinterpret_cast<const MT*>(dt.M) + dt.moff[s];
  const XT* __restrict__ gs = g + voff;
  const int c = it.y + 2 * threadIdx.x;
  const int rbeg = max(it.z, it.y), rend = min(it.z + kTChunk, n);
  double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
  if (c < n) {
    const bool two = c + 1 < n;
    int i = rbeg;
    for (; i + 1 < rend; i += 2) {
      const double g0 = (double)gs[i], g1 = (double)gs[i + 1];
      const MT* r0p = M + (long)i * dense_ld(n) + c;
      const MT* r1p = r0p + dense_ld(n);
      a0 += (double)r0p[0] * g0;
      b0 += (double)r1p[0] * g1;
      if (two) {
        a1 += (double)r0p[1] * g0;
        b1 += (double)r1p[1] * g1;
      }
    }
    if (i < rend) {
      const double g0 = (double)gs[i];
      const MT* r0p = M + (long)i * dense_ld(n) + c;
      a0 += (double)r0p[0] * g0;
      if (two) a1 += (double)r0p[1] * g0;
    }
  }
  double* part = dt.part + (long)it.w * kTCols;
  part[2 * threadIdx.x] = a0 + b0;
  part[2 * threadIdx.x + 1] = a1 + b1;
}

// y = T^{-T} g from the partial sums: item (system, c0, first slot, slots), slots in
// row-chunk order.
template <typename XT>
__global__ __launch_bounds__(kNT) void gemv_lower_t_sum_kernel(DenseTriDev dt, XT* __restrict__ y,
                                                               const int* __restrict__ done) {
  if (done && *done) return;
  const int4 it = dt.red[blockIdx.x];
  const int s = it.x;
  const int n = dt.n[s];
  for (int c = threadIdx.x; c < kTCols; c += kNT) {
    if (it.y + c >= n) break;
    double acc = 0.0;
    for (int k = 0; k < it.w; ++k) acc += dt.part[(long)(it.z + k) * kTCols + c];
    y[dt.voff[s] + it.y + c] = (XT)acc;
  }
}

}  // namespace

void dense_row_items(int sys, int n, std::vector<int4>& items) {
  const int m = (n + kHalfRows - 1) / kHalfRows;  // groups of four rows, the last one ragged
  for (int k = 0; k < (m + 1) / 2; ++k) {
    const int a0 = k * kHalfRows, na = std::min(kHalfRows, n - a0);
    const int kb = m - 1 - k;
    int b0 = 0, nb = 0;
    if (kb > k) {
      b0 = kb * kHalfRows;
      nb = std::min(kHalfRows, n - b0);
    }
    items.push_back(make_int4(sys, a0, b0, na | (nb << 4)));
  }
}

// Steps per batch for a launch whose largest system has n rows: an item's list holds
// about (n + 4) / W vectors (its two groups' columns), and a batch of D steps plus the
// same-batch tail takes (D + 1) x 256 of them; the fewest steps that cover the list in
// one batch, at most row_steps (larger systems take several batches).
template <typename T>
static int row_steps_for(int n) {
  constexpr int W = 16 / (int)sizeof(T);
  const int len = n > 0 ? (n + 4 + W - 1) / W : 1 << 30;
  int d = 1;
  while (d < row_steps<T>() && (d + 1) * kNT < len) d *= 2;
  return d;
}

template <bool UP, typename T, int D>
static void rows_launch_d(hipStream_t s, const DenseTriDev& dt, const void* f, void* y, const int* done,
                          hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0 && ev1)
    hipExtLaunchKernelGGL(gemv_tri_rows_kernel<UP, T, T, D>, dim3(dt.nitem_n), dim3(kNT), 0, s, ev0, ev1, 0, dt,
                          (const T*)f, (T*)y, done);
  else
    gemv_tri_rows_kernel<UP, T, T, D><<<dt.nitem_n, kNT, 0, s>>>(dt, (const T*)f, (T*)y, done);
}

// One row-product launch; with events, the dispatch itself stamps its start and end
// into them (measurement only).
template <bool UP, typename T>
static void rows_launch(hipStream_t s, const DenseTriDev& dt, const void* f, void* y, const int* done,
                        hipEvent_t ev0, hipEvent_t ev1) {
  const int d = row_steps_for<T>(dt.one_n > 0 ? dt.one_n : dt.max_n);
  if (d == 1) rows_launch_d<UP, T, 1>(s, dt, f, y, done, ev0, ev1);
  else if (d == 2) rows_launch_d<UP, T, 2>(s, dt, f, y, done, ev0, ev1);
  else if (d == 4) rows_launch_d<UP, T, 4>(s, dt, f, y, done, ev0, ev1);
  else rows_launch_d<UP, T, row_steps<T>()>(s, dt, f, y, done, ev0, ev1);
}

void launch_dense_lower(hipStream_t s, const DenseTriDev& dt, bool mfp32, bool xfp32, const void* f, void* y,
                        const int* done, hipEvent_t ev0, hipEvent_t ev1) {
  if (dt.nitem_n <= 0) return;
  if (mfp32 && xfp32) rows_launch<false, float>(s, dt, f, y, done, ev0, ev1);
  else rows_launch<false, double>(s, dt, f, y, done, ev0, ev1);
}

void launch_dense_lower_t(hipStream_t s, const DenseTriDev& dt, bool mfp32, bool xfp32, const void* g, void* y,
                          const int* done, hipEvent_t ev0, hipEvent_t ev1) {
  if (dt.MT) {  // stored transpose: row products of the upper-triangular T^{-T}
    if (dt.nitem_n <= 0) return;
    if (mfp32 && xfp32) rows_launch<true, float>(s, dt, g, y, done, ev0, ev1);
    else rows_launch<true, double>(s, dt, g, y, done, ev0, ev1);
    return;
  }
  if (ev0) (void)hipEventRecord(ev0, s);  // two kernels: events around both
  if (dt.nitem_t > 0) {
    if (mfp32 && xfp32) {
      gemv_lower_t_part_kernel<float, float><<<dt.nitem_t, kNT, 0, s>>>(dt, (const float*)g, done);
      gemv_lower_t_sum_kernel<float><<<dt.nred, kNT, 0, s>>>(dt, (float*)y, done);
    } else {
      gemv_lower_t_part_kernel<double, double><<<dt.nitem_t, kNT, 0, s>>>(dt, (const double*)g, done);
      gemv_lower_t_sum_kernel<double><<<dt.nred, kNT, 0, s>>>(dt, (double*)y, done);
    }
  }
  if (ev1) (void)hipEventRecord(ev1, s);
}

void launch_transpose(hipStream_t s, int n, const void* X, void* Y, bool fp32) {
  const dim3 grid((n + 31) / 32, (n + 31) / 32);
  if (fp32) transpose_kernel<float><<<grid, kNT, 0, s>>>(n, (const float*)X, (float*)Y);
  else transpose_kernel<double><<<grid, kNT, 0, s>>>(n, (const double*)X, (double*)Y);
}

bool dense_tri_inverse(hipStream_t s, int n, int voff, const int* rp, const int* ci, const double* v, double* M,
                       double* work, std::string* msg) {
  const long ld = dense_ld(n);
  bool ok = hipMemsetAsync(M, 0, sizeof(double) * (size_t)n * ld, s) == hipSuccess;
  if (ok) {
    scatter_lower_kernel<<<std::min((n + kNT - 1) / kNT, 1024), kNT, 0, s>>>(n, voff, rp, ci, v, M);
    leaf_inverse_kernel<<<(n + kLeaf - 1) / kLeaf, kLeaf, 0, s>>>(n, M);
    ok = hipGetLastError() == hipSuccess;
  }
  // merge inverted spans, all pairs of one span length in one launch per product: pair z
  // starts at row a = 2 sp z; A = rows/columns [a, a+sp), C = [a+sp, e), off-diagonal
  // block B = M[a+sp:e, a:a+sp]; W = B A^{-1} into work (pair z at z sp^2, row stride
  // sp), then B = -C^{-1} W. Only the last pair can be shorter (e = n).
  for (int sp = kLeaf; ok && sp < n; sp *= 2) {
    const int nm = (n - sp + 2 * sp - 1) / (2 * sp);  // pairs: a + sp < n
    const int a_last = (nm - 1) * 2 * sp;
    const int m2_last = std::min(a_last + 2 * sp, n) - a_last - sp;
    const int m2 = nm > 1 ? sp : m2_last;
    const long stride = 2L * sp * (ld + 1);
    double* B0 = M + (long)sp * ld;
    ok = launch_dgemm_batched(s, B0, stride, (int)ld, M, stride, (int)ld, work, (long)sp * sp, sp, m2, m2_last, sp,
                              sp, sp, nm, 1.0);
    ok = ok && launch_dgemm_batched(s, B0 + sp, stride, (int)ld, work, (long)sp * sp, sp, B0, stride, (int)ld, m2,
                                    m2_last, m2, m2_last, sp, nm, -1.0);
  }
  if (!ok && msg && msg->empty()) *msg = "dense triangular inverse failed";
  return ok;
}

void launch_to_type(hipStream_t s, long n, const double* a, void* y, bool fp32) {
  const int grid = (int)std::min<long>((n + kNT - 1) / kNT, 4096);
  if (fp32) to_type_kernel<float><<<grid, kNT, 0, s>>>(n, a, (float*)y);
  else to_type_kernel<double><<<grid, kNT, 0, s>>>(n, a, (double*)y);
}

}  // namespace cpc
