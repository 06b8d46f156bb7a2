// Internal interface between the solver and the allocation-free entry point
// (noalloc.hip): the device memory a PCG solve uses beyond its vectors and matrices.
#pragma once

#include "../../include/cpc.h"
#include "kernels.hpp"

namespace cpc {

// Device pointers of a solve's scratch: the PCG scalars and reduction arrival
// counters, the per-workgroup partial sums of the reductions (kPartials doubles) and
// the three counters of the level-scheduled sweeps (ticket, exited, error flag).
struct SolveScratch {
  PcgState* st;
  double* partials;
  SweepSync sync;
};

// Records msg as the message cpc_last_error() returns and passes st through.
cpc_status fail(cpc_status st, const char* msg);
int handle_device(const cpc_solver* h);
bool handle_is_batch(const cpc_solver* h);
cpc_status run_solve_on_scratch(cpc_solver* h, const double* b, double* x, int use_x0, double tol, int maxit,
                                int32_t* iters, double* relres, const SolveScratch& sc);

}  // namespace cpc
