// Host-side SETUP of the combined preconditioner: input validation, ILU(0)
// factorisation, classical Ruge-Stueben coarsening and interpolation, sweep
// schedules for the level-scheduled triangular kernels, and the exact coarsest
// solve. Everything here runs once per cpc_setup.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace cpc {

struct HostCsr {
  int n = 0;      // rows
  int ncols = 0;  // columns
  std::vector<int> rp, ci;
  std::vector<double> v;
  int64_t nnz() const { return rp.empty() ? 0 : rp[n]; }
};

// Input contract of cpc_setup. Returns a cpc_status value; msg gets the reason.
int validate_csr(int n, const int32_t* rp, const int32_t* ci, const double* v, bool check_symmetry,
                 std::string* msg);

// ILU(0) (Algorithm 3.1 with level of fill 0): values on the pattern of A,
// strictly lower part = L (unit diagonal implied), rest = U. Returns cpc_status.
int ilu0_factor(const HostCsr& a, std::vector<double>& lu, std::string* msg);

// ILU(k) by levels of fill (Algorithm 3.1): f holds the kept pattern (sorted rows) with
// L strictly lower (unit diagonal implied) and U on and above the diagonal; lev the
// level of fill of each kept entry. k = 0 gives the pattern of a and ilu0_factor's
// values. CPC_E_NOT_SPD on a pivot <= 0.
int iluk_factor(const HostCsr& a, int k, HostCsr& f, std::vector<int>& lev, std::string* msg);

// Classical C/F splitting (1 = C, 0 = F). Returns the number of C points.
int rs_coarsen(const HostCsr& a, double theta, std::vector<int>& cf);

// Classical Ruge-Stueben interpolation for the splitting cf: P has a.n rows and
// nc columns. Returns false on allocation failure.
bool rs_interpolation(const HostCsr& a, double theta, const std::vector<int>& cf, int nc, HostCsr& P);

// Explicit transpose (R = P^T).
HostCsr transpose(const HostCsr& a);

// Schedule of one sweep direction over a matrix: rows are cut into contiguous
// blocks of R rows; each block is processed by one workgroup in the order of its
// own (block-local) level sets; a block waits on per-block progress counters of
// earlier blocks (later blocks for the backward direction) before a level whose
// rows depend on them.
struct SweepSchedule {
  int n = 0, R = 0, nblk = 0;  // R: largest block
  bool forward = true;
  std::vector<int> blk_row;   // nblk+1: first row of each block
  std::vector<int> perm;      // rows in processing order, block after block in processing order
  std::vector<int> blk_beg;   // nblk: first global level of block b (b in row order)
  std::vector<int> blk_end;   // nblk: one past the last global level of block b
  std::vector<int> lvl_ptr;   // nlev+1: range of perm of each global level
  std::vector<int> wait_ptr;  // nlev+1: range of the wait list of each global level
  std::vector<int> wait_blk;  // block to wait on
  std::vector<int> wait_need; // progress value (levels completed) that block must reach
  std::vector<int> publish;   // nlev: 1 if some block waits for this level's completion
  int global_depth = 0;       // number of level sets of the whole dependency graph
  int max_local_levels = 0;
  int64_t max_level_entries = 0;  // most dependency entries of one level with two or more rows
};

// Build the schedule of the lower (forward) or upper (backward) sweep of a with
// blocks of at most R rows. Block boundaries are moved back (by at most R/2) to a
// row that is not coupled to the row before it, so that a block's first rows do not
// depend on the last (deepest) rows of the previous block. With max_entries > 0, a
// level whose rows hold more dependency entries (entries left of the diagonal for the
// forward direction, right of it for the backward one) is cut into consecutive levels
// of at most max_entries entries each; a single row longer than that forms a level of
// its own.
SweepSchedule build_sweep(const HostCsr& a, bool forward, int R, int64_t max_entries = 0);

// Block starts used by build_sweep (size nblk + 1, last = n).
std::vector<int> sweep_block_starts(const HostCsr& a, int R);

// Depth of the lower-triangular dependency graph (number of level sets).
int lower_depth(const HostCsr& a);

// Dense inverse of an SPD matrix via its Cholesky factor (row-major n x n).
// Returns cpc_status (CPC_E_NOT_SPD when a pivot is not positive).
int dense_spd_inverse(const HostCsr& a, std::vector<double>& inv, std::string* msg);

}  // namespace cpc
