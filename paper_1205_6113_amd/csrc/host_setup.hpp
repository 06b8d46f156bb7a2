// Host-side SETUP of the combined preconditioner: input validation, ILU(0)
// factorisation, classical Ruge-Stueben coarsening and interpolation, sweep
// schedules for the level-scheduled triangular kernels, and the exact coarsest
// solve. Everything here runs once per cpc_setup.
#pragma once

#include <cstdint>
#include <string>
#include <algorithm>
#include <memory>
#include <thread>
#include <utility>
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
// its own. parts (optional, {0, ..., n}): row ranges that no block may span (the
// systems of a batch); every part boundary is a block boundary.
SweepSchedule build_sweep(const HostCsr& a, bool forward, int R, int64_t max_entries = 0,
                          const std::vector<int>* parts = nullptr);

// Schedule of the one-wave triangular-solve kernel. Rows are cut into blocks that are
// unions of up to M segments of W rows spaced `stride` rows apart: row i lies in the
// group i / (stride * M) and the segment (i % stride) / W of it (M = 1: contiguous
// blocks of W rows). On a grid in natural order, the stride is the longest coupling
// (one plane of a 3-D grid), so the couplings between consecutive planes of a group
// stay inside a block instead of crossing to another block. Blocks are processed in
// a topological order of their dependency graph (the schedule is refused when that
// graph has a cycle); within a block the rows run in order of their global depth
// (the level sets of the whole solve), each row at an LDS slot of its own.
struct WaveSchedule {
  bool forward = true;
  int n = 0, nblk = 0, R = 0;  // R: most rows of one block
  int W = 0, M = 1, stride = 0;
  int global_depth = 0;
  std::vector<int> blk_ptr;   // nblk + 1: rows of the t-th processed block in `rows`
  std::vector<int> rows;      // the rows of each block in (depth, row) order
  std::vector<int> blk_lvl;   // nblk + 1: levels of block t in lvl_ptr
  std::vector<int> lvl_ptr;   // level boundaries within `rows`
  std::vector<int> slot;      // [n] LDS slot of each row within its block
  std::vector<int> block_of;  // [n] processing index of each row's block
  std::vector<int> blk_part;  // nblk: part (system) of block t (build_wave_schedule_parts)
};

// Longest lower coupling i - j (j < i) that most rows share (0 for a diagonal matrix).
int dominant_stride(const HostCsr& a);

// Returns false when the blocks' dependency graph has a cycle.
bool build_wave_schedule(const HostCsr& a, bool forward, int W, int M, int stride, WaveSchedule& s);

// The same for a block-diagonal matrix whose diagonal blocks are the row ranges
// [parts[p], parts[p+1]) (the systems of a batch; {0, n} for one system): each part
// gets its own schedule with its own dominant coupling distance (contiguous blocks
// where its segmented blocks would form a cycle), built on up to `threads` host
// threads, and the parts' blocks are merged in an interleaved order (blocks of
// different parts are independent). Always succeeds.
void build_wave_schedule_parts(const HostCsr& a, bool forward, int W, int M, const std::vector<int>& parts,
                               int threads, WaveSchedule& s);

// One-wave form of a triangular solve over a wave schedule (the layout the kernel
// reads): each level of each block cut into steps of G = 64 / tb rows, a row's
// dependency entries dealt over its tb lanes (entry e on lane e % tb at position
// e / tb of the step's [k][64] arrays), padding entries with column R (a slot that
// holds zero) and value 0, padding groups with row -1. Columns: the slot of j inside
// the row's block, -(j + 1) outside. (tb, k) is the shape from `shapes` that holds the
// longest row in the fewest steps (then the smallest k).
// fn(lo, hi) over [0, count) cut into contiguous chunks of at least `grain` items, on
// up to `threads` host threads (fn must not throw).
template <typename F>
void chunked(int64_t count, int threads, int64_t grain, F fn) {
  threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, count / std::max<int64_t>(grain, 1) + 1));
  if (threads == 1) {
    fn((int64_t)0, count);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&, t] { fn(count * t / threads, count * (t + 1) / threads); });
  for (auto& th : pool) th.join();
}

// Allocator whose resize leaves new elements uninitialised: the large pack arrays are
// then first touched by the threads that fill them (page faults in parallel).
template <typename T>
struct NoInitAlloc : std::allocator<T> {
  using value_type = T;
  template <typename U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <typename U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <typename U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <typename U, typename... Args>
  void construct(U* p, Args&&... args) {
    ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
  }
};
template <typename T>
using RawVec = std::vector<T, NoInitAlloc<T>>;

struct WavePack {
  int tb = 0, k = 0, nblk = 0, R = 0;
  int64_t nsteps = 0;
  std::vector<int> blk_step;  // nblk + 1, processing order
  RawVec<int> row;            // nsteps * (64 / tb)
  RawVec<int> slot;           // nsteps * (64 / tb), LDS slot of the row
  RawVec<double> dinv;        // nsteps * (64 / tb), reciprocal diagonal (0 for padding)
  RawVec<int> col;            // nsteps * k * 64
  RawVec<double> val;         // nsteps * k * 64
};

// Returns false (w untouched) when no shape holds the longest row. Built on up to
// `threads` host threads (blocks fill disjoint ranges).
bool build_wave_pack(const HostCsr& a, const std::vector<double>& vals, const WaveSchedule& s,
                     const std::vector<std::pair<int, int>>& shapes, WavePack& w, int threads = 1);

// Block starts used by build_sweep (size nblk + 1, last = n).
std::vector<int> sweep_block_starts(const HostCsr& a, int R, const std::vector<int>* parts = nullptr);

// Depth of the lower-triangular dependency graph (number of level sets).
int lower_depth(const HostCsr& a);

// Dense inverse of an SPD matrix via its Cholesky factor (row-major n x n).
// Returns cpc_status (CPC_E_NOT_SPD when a pivot is not positive).
int dense_spd_inverse(const HostCsr& a, std::vector<double>& inv, std::string* msg);

}  // namespace cpc
