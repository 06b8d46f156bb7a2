// cpc_solve_noalloc: the PCG solve of cpc_solve for callers that cannot allocate
// device memory. Its scratch (PCG scalars, reduction partials, sweep counters) lives
// in one file-scope device array per GPU, located once per device with
// hipGetSymbolAddress; the call itself allocates nothing and launches every
// iteration eagerly (instantiating a graph would allocate).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/cpc.h"
#include "kernels.hpp"
#include "solve_scratch.hpp"

namespace {

constexpr size_t kSlot = 256;
constexpr size_t kOffState = 0;
constexpr size_t kOffPartials = kSlot;
constexpr size_t kOffTicket = kOffPartials + sizeof(double) * cpc::kPartials;
constexpr size_t kOffExited = kOffTicket + kSlot;
constexpr size_t kOffErr = kOffExited + kSlot;
constexpr size_t kNeed = kOffErr + kSlot;
constexpr size_t kScratchBytes = 65536;  // the stated maximum (64 KiB per GPU)
static_assert(sizeof(cpc::PcgState) <= kSlot, "PCG state must fit its slot");
static_assert(kOffTicket % kSlot == 0, "counters start on their own slots");
static_assert(kNeed <= kScratchBytes, "the solve's scratch must fit the array");

// Device-side storage. In host code `scratch` names a host-side stand-in, never the
// device address: only the pointer hipGetSymbolAddress returned is passed on.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on `dev` (current), located on the first call.
hipError_t scratch_ptr(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" cpc_status cpc_solve_noalloc(cpc_handle h, const double* b_dev, double* x_dev, int32_t use_x0, double tol,
                                        int32_t maxit, int32_t* iters, double* relres) {
  if (!h) return cpc::fail(CPC_E_ARG, "null handle");
  if (cpc::handle_is_batch(h)) return cpc::fail(CPC_E_ARG, "batch handle: cpc_solve_noalloc solves single systems");
  if (kNeed > kScratchBytes) return cpc::fail(CPC_E_ARG, "solve scratch exceeds the 64 KiB static array");
  const int dev = cpc::handle_device(h);
  if (dev < 0 || dev >= kMaxDevices) return cpc::fail(CPC_E_ARG, "device index beyond the scratch table");
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return cpc::fail(CPC_E_DEVICE, "hipGetDevice failed");
  if (prev != dev && hipSetDevice(dev) != hipSuccess) return cpc::fail(CPC_E_DEVICE, "hipSetDevice failed");
  void* base = nullptr;
  hipError_t e = scratch_ptr(dev, &base);
  cpc_status st;
  if (e != hipSuccess) {
    st = cpc::fail(CPC_E_DEVICE, "hipGetSymbolAddress(scratch) failed");
  } else {
    unsigned char* p = static_cast<unsigned char*>(base);
    cpc::SolveScratch sc;
    sc.st = reinterpret_cast<cpc::PcgState*>(p + kOffState);
    sc.partials = reinterpret_cast<double*>(p + kOffPartials);
    sc.sync.ticket = reinterpret_cast<unsigned*>(p + kOffTicket);
    sc.sync.exited = reinterpret_cast<unsigned*>(p + kOffExited);
    sc.sync.err = reinterpret_cast<unsigned*>(p + kOffErr);
    // the array keeps the previous call's contents; run_solve_on_scratch clears the
    // sweep counters on the handle's stream before the first kernel
    st = cpc::run_solve_on_scratch(h, b_dev, x_dev, use_x0, tol, maxit, iters, relres, sc);
  }
  if (prev != dev) (void)hipSetDevice(prev);
  return st;
}
