// One-wave, barrier-free level-scheduled triangular solve: the forward (D+L) and
// (I+L) solves and the backward (D+U) solves of the Gauss-Seidel smoother and of
// ILU(0), evaluated exactly as the natural-order substitution they replace (only the
// order of each row's additions differs).
//
// A workgroup is one wave. It takes blocks of rows from a ticket counter in dependency
// order and walks each block in steps (up to 64 / TB rows of one level,
// TB lanes per row, K dependency entries per lane). Values of the block's own rows
// live in LDS; with a single wave, a value written to LDS in one step is visible to
// the next step's reads without a barrier (LDS instructions of one wave execute in
// order). Values of other blocks are read from the output vector, which starts filled
// with a sentinel bit pattern: a value that is not the sentinel is final, and a read
// that still finds the sentinel polls the address (bounded; past the limit the error
// flag is set) until the other block has stored it.
//
// The steps are stored in processing order, so the data of a step d places ahead sits
// at a computed address. The loop keeps a ring of D steps in registers: at each step
// it issues the entry data of the step D ahead and, for the step D2 ahead whose
// columns have arrived, the values it needs from other blocks and the right-hand side.
// Every step issues the same loads (steps past the end of a block read a valid dummy
// and write nothing), and no loop with memory loads sits in the step, so the waits the
// compiler places count exactly the loads still in flight instead of draining them.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "wave_sum.hpp"

namespace cpc {

namespace {

constexpr int kD = 8;   // steps of entry data in flight
constexpr int kD2 = 2;  // steps ahead at which other blocks' values and f are read

__device__ __forceinline__ bool w_sentinel(double v) {
  return (unsigned long long)__double_as_longlong(v) == kSentinel64;
}
__device__ __forceinline__ bool w_sentinel(float v) { return __float_as_uint(v) == kSentinel32; }

template <int K, typename VT, typename XT>
struct WSlot {
  int col[K];
  VT v[K];
  int row, slot;
  VT dinv;
  XT rem[K];  // values of other blocks' rows (the sentinel if not yet stored)
  XT fv, bv;
};

template <int OP, int TB, int K, typename VT, typename XT>
__global__ __launch_bounds__(64) void tri_wave_kernel(WaveDev w, const XT* __restrict__ f, XT* x,
                                                      const XT* __restrict__ base, XT* __restrict__ out,
                                                      SweepSync sy, const int* __restrict__ done, long spin_limit) {
  constexpr bool UNIT = (OP == SWEEP_UNIT_LOWER);
  constexpr bool OUT = (OP == SWEEP_UPPER_OUT);
  constexpr int G = 64 / TB;
  using S = WSlot<K, VT, XT>;
  extern __shared__ unsigned char w_smem[];
  XT* xs = reinterpret_cast<XT*>(w_smem);
  if (done && *done) return;  // before taking a ticket: the counters stay untouched
  const int lane = threadIdx.x;
  const int g = lane / TB;
  const bool lead = (lane % TB) == 0;
  const VT* __restrict__ wval = reinterpret_cast<const VT*>(w.val);
  const VT* __restrict__ wdinv = reinterpret_cast<const VT*>(w.dinv);
  if (lane == 0) xs[w.R] = XT(0);  // the padding entries' slot

  for (;;) {
    int t = 0;
    if (lane == 0) t = (int)atomicAdd(sy.ticket, 1u);
    t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
    if (t >= w.nblk) break;
    if (masked(w.mask, t)) continue;  // a block of a system that has stopped
    const int s0 = w.blk_step[t], s1 = w.blk_step[t + 1];

    // entry data, row and diagonal of step s (clamped to the block's last step: past
    // the end the addresses stay valid and the row is dropped)
    auto issue1 = [&](S& sl, int s) {
      const int sc = s < s1 ? s : s1 - 1;
      const size_t eb = (size_t)sc * (K * 64) + lane;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        sl.col[k] = w.col[eb + k * 64];
        sl.v[k] = wval[eb + k * 64];
      }
      const int r = w.row[(size_t)sc * G + g];
      sl.slot = w.slot[(size_t)sc * G + g];
      sl.row = s < s1 ? r : -1;
      if constexpr (!UNIT) sl.dinv = wdinv[(size_t)sc * G + g];
    };
    // values from other blocks (agent-scope loads: another block stores them), the
    // right-hand side and the base of the U-solve epilogue; dummy valid addresses
    // where there is nothing to read
    auto issue2 = [&](S& sl) {
      const int rw = sl.row >= 0 ? sl.row : 0;
      sl.fv = f[rw];
      if constexpr (OUT) sl.bv = base[rw];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int c = sl.col[k];
        const int j = c < 0 ? -(c + 1) : 0;
        sl.rem[k] = __hip_atomic_load(x + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    };
    auto poll = [&](XT v, int j) -> XT {
      long spins = 0;
      while (w_sentinel(v)) {
        if (++spins > spin_limit) {
          atomicOr(sy.err, 1u);
          return XT(0);
        }
        if ((spins & 255) == 0 && __hip_atomic_load(sy.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
          return XT(0);
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(x + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      return v;
    };
    auto compute = [&](S& sl) {
      bool wait = false;
#pragma unroll
      for (int k = 0; k < K; ++k) wait |= (sl.col[k] < 0) && w_sentinel(sl.rem[k]);
      if (__any(wait)) {
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (sl.col[k] < 0 && w_sentinel(sl.rem[k])) sl.rem[k] = poll(sl.rem[k], -(sl.col[k] + 1));
      }
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int c = sl.col[k];
        const double xl = (double)xs[c >= 0 ? c : w.R];
        const double xv = c >= 0 ? xl : (double)sl.rem[k];
        sum += (double)sl.v[k] * xv;
      }
      sum = gsum<TB>(sum);
      const double fv = (double)sl.fv;
      const double xi = UNIT ? fv - sum : (fv - sum) * (double)sl.dinv;
      if (lead && sl.row >= 0) {
        const XT xo = (XT)xi;
        xs[sl.slot] = xo;
        __hip_atomic_store(x + sl.row, xo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if constexpr (OUT) out[sl.row] = (XT)((double)sl.bv + (double)xo);
      }
    };

    S ring[kD];
#pragma unroll
    for (int d = 0; d < kD; ++d) issue1(ring[d], s0 + d);
#pragma unroll
    for (int d = 0; d < kD2; ++d) issue2(ring[d]);
    for (int s = s0; s < s1; s += kD) {
#pragma unroll
      for (int d = 0; d < kD; ++d) {
        compute(ring[d]);
        issue2(ring[(d + kD2) % kD]);
        issue1(ring[d], s + d + kD);
      }
    }
  }
  // the last workgroup to leave resets the counters for the next launch
  int last = 0;
  if (lane == 0) last = (atomicAdd(sy.exited, 1u) == gridDim.x - 1);
  if (__shfl(last, 0)) {
    if (lane == 0) {
      *sy.ticket = 0u;
      *sy.exited = 0u;
    }
  }
}

template <int OP, int TB, int K, typename VT, typename XT>
void launch_one(hipStream_t s, const WaveDev& w, const void* f, void* x, const void* base, void* out,
                const SweepSync& sync, const int* done, long spin_limit, hipEvent_t ev0, hipEvent_t ev1) {
  const int lds = wave_lds_bytes(w.R, sizeof(XT) == 4);
  static int attr = 65536;  // dynamic LDS the kernel may use without an attribute
  if (lds > attr) {
    if (hipFuncSetAttribute((const void*)tri_wave_kernel<OP, TB, K, VT, XT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess) {
      (void)hipGetLastError();  // leave no sticky error; the launch below reports the failure
    } else {
      attr = 160 * 1024;
    }
  }
  if (ev0 && ev1)  // measurement: the dispatch stamps its own start and end
    hipExtLaunchKernelGGL(tri_wave_kernel<OP, TB, K, VT, XT>, dim3(w.grid), dim3(64), lds, s, ev0, ev1, 0, w,
                          (const XT*)f, (XT*)x, (const XT*)base, (XT*)out, sync, done, spin_limit);
  else
    tri_wave_kernel<OP, TB, K, VT, XT><<<w.grid, 64, lds, s>>>(w, (const XT*)f, (XT*)x, (const XT*)base, (XT*)out,
                                                               sync, done, spin_limit);
}

template <int OP, typename VT, typename XT>
void dispatch(hipStream_t s, const WaveDev& w, const void* f, void* x, const void* base, void* out,
              const SweepSync& sync, const int* done, long spin_limit, hipEvent_t ev0, hipEvent_t ev1) {
#define CPC_WV(TB_, K_)                                                                    \
  if (w.tb == TB_ && w.k == K_) {                                                          \
    launch_one<OP, TB_, K_, VT, XT>(s, w, f, x, base, out, sync, done, spin_limit, ev0, ev1); \
    return;                                                                                \
  }
  CPC_WV(1, 2) CPC_WV(1, 4) CPC_WV(2, 2) CPC_WV(2, 4) CPC_WV(4, 2) CPC_WV(4, 4)
  CPC_WV(8, 2) CPC_WV(8, 4) CPC_WV(16, 2) CPC_WV(16, 4)
#undef CPC_WV
}

}  // namespace

bool wave_shape_supported(int tb, int k) {
  return (tb == 1 || tb == 2 || tb == 4 || tb == 8 || tb == 16) && (k == 2 || k == 4);
}

int wave_lds_bytes(int R, bool fp32) { return (R + 1) * (fp32 ? 4 : 8); }

void launch_wave_sweep(hipStream_t s, int op, const WaveDev& w, bool fp32, const void* f, void* x,
                       const void* base, void* out, const SweepSync& sync, const int* done, long spin_limit,
                       hipEvent_t ev0, hipEvent_t ev1) {
  if (w.nblk <= 0) return;
#define CPC_WOP(OPC)                                                                                     \
  if (fp32) dispatch<OPC, float, float>(s, w, f, x, base, out, sync, done, spin_limit, ev0, ev1);        \
  else dispatch<OPC, double, double>(s, w, f, x, base, out, sync, done, spin_limit, ev0, ev1);
  switch (op) {
    case SWEEP_LOWER: CPC_WOP(SWEEP_LOWER) break;
    case SWEEP_UPPER: CPC_WOP(SWEEP_UPPER) break;
    case SWEEP_UNIT_LOWER: CPC_WOP(SWEEP_UNIT_LOWER) break;
    default: CPC_WOP(SWEEP_UPPER_OUT) break;
  }
#undef CPC_WOP
}

}  // namespace cpc
