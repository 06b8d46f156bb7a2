// Device kernels of the SOLVE phase and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace cpc {

// Scalars of one PCG run, kept on the device so that no iteration needs the host.
// Entries of the PCG's partial-sum buffer: the grid of a last-workgroup reduction is at
// most this (two reductions of at most half of it share the buffer in the first step).
constexpr int kPartials = 4096;

struct PcgState {
  double rz;      // <r, z> of the current iterate
  double pq;      // <p, A p>
  double alpha, beta;
  double rr;      // ||r||^2
  double bb;      // ||b||^2
  double tol;     // relative residual tolerance
  double relres;  // ||r|| / ||b||
  int iters;      // completed iterations
  int maxit;
  int done;       // 0 running, 1 converged, 2 iteration cap, 3 breakdown, 4 zero right-hand side
  int pad;
  unsigned cnt[8];  // arrival counters of the last-workgroup reductions (reset by that workgroup)
};

enum { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_MAXIT = 2, DONE_BREAKDOWN = 3, DONE_ZERO_RHS = 4 };

// Per-system mask of a batched solve: unit k of a launch (a row, a block, a system of a
// dense list) belongs to system of[k] (-1: to none alone), and the launch skips units
// whose system has stopped (done[s] != 0). Null done: no mask. Units are masked only where
// no unit of a running system waits on them (blocks never span two systems).
struct SysMask {
  const int* of = nullptr;
  const int* done = nullptr;
};
__device__ __forceinline__ bool masked(const SysMask& m, int k) {
  if (!m.done || !m.of) return false;
  const int s = m.of[k];
  return s >= 0 && m.done[s] != 0;
}

// Device counters shared by every persistent sweep launch (self-resetting).
struct SweepSync {
  unsigned* ticket;  // [1]
  unsigned* exited;  // [1]
  unsigned* err;     // [1] set when a wait for another block's row exceeded its bound
};

// Not-yet-solved marker of a sweep's output: signalling-NaN bit patterns, which no
// arithmetic result takes (arithmetic only produces quiet NaNs).
constexpr unsigned long long kSentinel64 = 0x7FF4DEADBEEF0001ull;
constexpr unsigned kSentinel32 = 0x7FA5DEADu;

// One level-scheduled triangular solve (see SweepSchedule in host_setup.hpp).
struct SweepDev {
  int n, R, nblk, nlev;  // R: rows of the largest block
  const int* blk_row;    // nblk + 1 row starts of the blocks
  const int* blk_beg;    // first level of each block
  const int* blk_end;
  const int* lvl_ptr;    // level -> first position in processing order
  int pcap;              // product slots per workgroup (largest entry count of a level with two or more rows)
  int maxl;              // most levels of one block
  int lds;               // dynamic LDS bytes of one workgroup
  int off_xs, off_rows, off_ptr, off_meta;  // byte offsets of the LDS arrays (products start at 0)
  int grid;              // workgroups launched
  int nt;                // threads per workgroup: 64 or 256
  SysMask mask{};        // by block (blocks within one system only)
};

enum SweepOp {
  SWEEP_LOWER = 0,       // x = (D+L)^{-1} f                         (forward)
  SWEEP_UPPER = 1,       // x = (D+U)^{-1} f                         (backward)
  SWEEP_UNIT_LOWER = 2,  // x = (I+L)^{-1} f                         (forward)
  SWEEP_UPPER_OUT = 3    // x = (D+U)^{-1} f, out = base + x         (backward)
};

struct MatDev {  // CSR on the device; values of type T
  int n;
  const int* rp;
  const int* ci;
  const int* dpos;  // position of the diagonal in each row (square matrices)
  const void* v;
  bool fp32;
  int steps;  // entries per lane a small launch takes at once in a row product: 1, 2 or 4
  // SpMV only: row k of the matrix is level row rid[k] of f and y (null: row k itself)
  const int* rid = nullptr;
  SysMask mask{};  // SpMV only: by level row (the output index)
};

// ---- launchers (all asynchronous on `s`) -----------------------------------
// y = A x (mode 0), y = f - A x (mode 1), y += A x (mode 2). xf32/ff32/yf32 select
// FP32 storage of x, f and y. Supported: all FP64; all FP32 (FP32 matrix); FP64
// matrix with FP32 x and y and FP64 f. Returns false for other combinations.
bool launch_spmv(hipStream_t s, const MatDev& A, int mode, const void* x, bool xf32, const void* f, bool ff32,
                 void* y, bool yf32, int tpr, const int* done);

// PCG: q = A p and <p, q>; the last workgroup sets pq, alpha (or flags breakdown).
void launch_spmv_pq(hipStream_t s, const MatDev& A, const double* p, double* q, double* partials, PcgState* st,
                    int tpr);
// x += alpha p, r -= alpha q, ||r||^2 -> relres, iteration count, convergence flag.
void launch_update_xr(hipStream_t s, int n, double* x, double* r, const double* p, const double* q,
                      double* partials, PcgState* st);
// <r, z> -> beta = rz_new / rz (first = true: rz only, and p = z).
void launch_dot_rz(hipStream_t s, int n, const double* r, const double* z, double* p, double* partials,
                   PcgState* st, bool first);
// p = z + beta p.
void launch_update_p(hipStream_t s, int n, const double* z, double* p, PcgState* st);
// Start of a solve: r = b - A x (use_x0) or r = b, x = 0; ||b||, ||r|| and the
// tolerance test before the first iteration.
void launch_pcg_init(hipStream_t s, const MatDev& A, const double* b, double* x, double* r, int use_x0,
                     double* partials, PcgState* st, int tpr);

// Per-system PCG scalars of a batch of independent systems (batch.hip). Rows of the
// concatenated vectors are cut into chunks that never straddle two systems.
struct BatchDev {
  int nsys, nchunks;
  const int* chunk_sys;  // [nchunks] system of each chunk
  const int* chunk_row;  // [nchunks+1] first row of each chunk
  const int* sys_chunk;  // [nsys+1] chunk range of each system
  double* partials;      // [4 * nchunks] one partial per chunk and reduction slot
  unsigned* cnt;         // [4 * nsys] arrival counters (reset by the last chunk)
  double *rz, *pq, *alpha, *beta, *rr, *bb, *relres;  // [nsys]
  int* iters;            // [nsys]
  int* done;             // [nsys] 0 running, else a DONE_* code
  const double* tol_dev; // relative residual tolerance (device scalar)
  const int* maxit_dev;  // iteration cap (device scalar)
};

// Dense solves e = inv f on segments of a level vector (coarsest systems of a depth).
struct DenseListDev {
  int nblk;               // workgroups (4 rows each)
  const int* blk_entry;   // [nblk] entry of each workgroup
  const int* blk_row0;    // [nblk] first row of each workgroup within its entry
  const int* n;           // [entries] rows of each system's coarsest matrix
  const int* off;         // [entries] offset of its segment in the level vector
  const long* inv_off;    // [entries] offset of its row-major inverse in inv
  const double* inv;      // concatenated inverses (FP64)
  SysMask mask{};         // by entry
};

void launch_bspmv_pq(hipStream_t s, const BatchDev& bd, const MatDev& A, const double* p, double* q, int tpr);
void launch_bupdate_xr(hipStream_t s, const BatchDev& bd, double* x, double* r, const double* p, const double* q);
void launch_bdot_rz(hipStream_t s, const BatchDev& bd, const double* r, const double* z, double* p, bool first);
void launch_bupdate_p(hipStream_t s, const BatchDev& bd, const double* z, double* p);
void launch_binit(hipStream_t s, const BatchDev& bd, const double* b, double* x, double* r);
void launch_bdense(hipStream_t s, const DenseListDev& dl, const void* f, void* e, bool fp32, const int* done);

// Rows of one triangular solve packed in processing order (see sweep.hip).
// One-wave form of a triangular solve (wave_sweep.hip; schedule and layout in
// host_setup.hpp, WaveSchedule / WavePack). The rows of each block are processed in
// steps: a step holds up to G = 64 / tb rows of one level (rows of a level are
// independent), each row on tb lanes, each lane holding k of the row's dependency
// entries. Steps are stored in processing order, block after block, so the data of the
// step d places ahead lies at a computed address.
struct WaveDev {
  int ok;               // 1 when the pack has this form
  int tb, k;            // lanes per row, entries per lane (a row holds at most tb * k entries)
  int nblk, R;          // blocks; LDS slots R + 1 (slot R holds zero, the padding entries' column)
  int nsteps;
  int grid;             // workgroups (one wave each) launched
  int W, M;             // segment width and segments per block of the schedule (for reports)
  const int* blk_step;  // [nblk + 1] steps of the t-th processed block: [blk_step[t], blk_step[t+1])
  const int* col;       // [nsteps][k][64] entry column: the slot of j within the row's block,
                        // -(j + 1) in another block, R for padding; entry e of a row on lane
                        // e % tb at position e / tb
  const void* val;      // [nsteps][k][64] entry values (0 for padding)
  const int* row;       // [nsteps][G] row of each group, -1 for none
  const int* slot;      // [nsteps][G] LDS slot of the group's row within its block
  const void* dinv;     // [nsteps][G] reciprocal diagonal of the group's row
  SysMask mask{};       // by ticket (processing position of the block)
};

struct SweepPackDev {
  WaveDev wave{};    // the one-wave form, used when wave.ok
  const int* row;    // [n] row of the p-th processed row
  const int* ptr;    // [n+1] dependency entries of processed row p: [ptr[p], ptr[p+1])
  const int* col;    // entry column: j - (first row of the block) for a column in the row's own
                     // block, -(j + 1) for a column in another block
  const void* val;   // entry values (FP64 or FP32)
  const void* diag;  // [n] reciprocal diagonal of processed row p (unused by the unit lower solve)
  int tb;            // lanes that sum one row's products
};

// Dense explicit inverses T^{-1} = (D+L)^{-1} of the systems of one level (dense_tri.hip).
constexpr int kTCols = 512;    // columns of one item of the transposed product
constexpr int kTChunk = 1024;  // rows of one item of the transposed product
constexpr int kHalfRows = 4;  // rows of one group of a row-product item (two groups per item)
struct DenseTriDev {
  const int* n;        // [nsys] rows of each system
  const long* moff;    // [nsys] element offset of each system's row-major inverse (row stride dense_ld(n))
  const int* voff;     // [nsys] first row of each system in the level vector
  const void* M;       // the inverses (lower triangular; FP64 or FP32)
  const void* MT;      // their transposes (upper triangular), or null: transposed product by items
  int nitem_n;         // row-product items: {system, first row of group A, of group B, rows of A | rows of B << 4}
  const int4* item_n;
  int nitem_t;         // partial sums of y = T^{-T} g: {system, first column, first row, slot}
  const int4* item_t;
  int nred;            // column sums of the partials: {system, first column, first slot, slots}
  const int4* red;
  double* part;        // [slots][kTCols]
  // A launch over one system (a diagonal block of the block-dense form, or a level held
  // whole): one_n > 0 gives its rows, its first row in the level vector and the offset
  // of its inverse, and the row items follow from the block index (the items of
  // dense_row_items), so the kernel reads no item or system entry before the inverse.
  int one_n;
  int one_voff;
  long one_moff;
  int one_sys;     // the system index (of mask) of a one_n launch
  int max_n = 0;   // rows of the launch's largest system (0: unknown), for the product's steps per batch
  SysMask mask{};  // by system index of the list (a block of the block-dense form)
};
// Row stride of a stored n x n inverse: n rounded up to a multiple of 4 elements, so
// that every row starts 16-byte aligned (the padding columns hold zeros), and 8 more
// when that is a multiple of 512: rows of a power-of-two system (the 4096-row blocks)
// then do not all start at one offset modulo the memory interleave (in a standalone test
// of 4096-row products the 64-byte pad saved 0.5 us of 13.7 per launch; larger pads did
// not). At most 16392 for the 16384-row limit, so a system's inverse stays within 32-bit
// byte offsets.
__host__ __device__ inline int dense_ld(int n) {
  const int l = (n + 3) & ~3;
  return l % 512 == 0 ? l + 8 : l;
}
// T^{-1} of rows [voff, voff + n) of the level CSR (columns offset by voff) into the
// dense n x dense_ld(n) array M (FP64), using work (>= the largest off-diagonal product).
bool dense_tri_inverse(hipStream_t s, int n, int voff, const int* rp, const int* ci, const double* v, double* M,
                       double* work, std::string* msg);
// Row-product items of one system of n rows (system index sys), appended to items:
// groups of four rows from the top paired with the mirrored groups from the bottom.
void dense_row_items(int sys, int n, std::vector<int4>& items);
// y = T^{-1} f and y = T^{-T} g through the stored inverse. ev0 / ev1 (measurement
// only): events stamped with the start and end of the dispatch.
void launch_dense_lower(hipStream_t s, const DenseTriDev& dt, bool mfp32, bool xfp32, const void* f, void* y,
                        const int* done, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void launch_dense_lower_t(hipStream_t s, const DenseTriDev& dt, bool mfp32, bool xfp32, const void* g, void* y,
                          const int* done, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void launch_to_type(hipStream_t s, long n, const double* a, void* y, bool fp32);
// O[z] = alpha * L[z] R[z] (FP64, row-major, matrix cores) for z < nb: L[z] rows x inner
// (row stride ldl), R[z] inner x cols (ldr), O[z] rows x cols (ldo); entry z's operands
// start z * sl, z * sr, z * so elements after entry 0's; the last entry has rows_last
// rows and inner_last inner indices. O[z] must not overlap any operand. Returns false
// on invalid sizes or a failed launch (dense_gemm.hip).
bool launch_dgemm_batched(hipStream_t s, const double* L, long sl, int ldl, const double* R, long sr, int ldr,
                          double* O, long so, int ldo, int rows, int rows_last, int inner, int inner_last, int cols,
                          int nb, double alpha);
void launch_transpose(hipStream_t s, int n, const void* X, void* Y, bool fp32);

// Persistent block-pipelined triangular solve over packed rows (sweep.hip). x must
// hold the sentinel in rows [0, sw.n) (launch_fill_sentinel) when it starts.
void launch_sweep_packed(hipStream_t s, int op, const SweepDev& sw, const SweepPackDev& pk, bool fp32,
                         const void* f, void* x, const void* base, void* out, const SweepSync& sync,
                         const int* done, long spin_limit);
void launch_fill_sentinel(hipStream_t s, int n, void* x, bool fp32, const int* done);
// The same triangular solves through the one-wave form of the pack (pk.wave.ok);
// x must hold the sentinel in every row of the system when it starts.
void launch_wave_sweep(hipStream_t s, int op, const WaveDev& w, bool fp32, const void* f, void* x,
                       const void* base, void* out, const SweepSync& sync, const int* done, long spin_limit,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Supported (lanes per row, entries per lane) of the one-wave form.
bool wave_shape_supported(int tb, int k);
int wave_lds_bytes(int R, bool fp32);
int sweep_max_rows_per_block();
int sweep_lds_budget();      // dynamic LDS bytes a sweep workgroup may use
int sweep_threads();         // threads per sweep workgroup

// e = inv f with a dense row-major inverse (coarsest level, FP64).
void launch_dense_matvec(hipStream_t s, int n, const double* inv, const void* f, bool ff32, void* e, bool ef32,
                         const int* done);

// Elementwise: z = a + b (op 0), y += a (op 1), y = a (op 2, copy), y = 0 (op 3),
// with optional FP32 storage of each operand.
void launch_vec(hipStream_t s, int op, int n, const void* a, bool af32, const void* b, bool bf32, void* y,
                bool yf32, const int* done);

// g[p] = -lam[i] * x[j] for every entry p = (i, j) of A.
void launch_neg_outer(hipStream_t s, const MatDev& A, const double* lam, const double* x, double* g);

// FP64 -> FP32 copy of a value array.
void launch_to_f32(hipStream_t s, int64_t n, const double* a, float* y);

// Galerkin product C = X * Y with the canonical accumulation order (see rap.hip).
// Symbolic: counts[i] = distinct columns of row i, or -1 for a row with more distinct
// columns than the LDS table holds (a wide row; the flag `wide` is then set). Numeric:
// rows with at least spgemm_table_capacity() entries in crp are left to the wide-row
// kernels; a mismatch with crp sets `overflow`.
void launch_spgemm_count(hipStream_t s, int nrows, const int* xrp, const int* xci, const int* yrp, const int* yci,
                         int* counts, int* wide);
void launch_spgemm_fill(hipStream_t s, int nrows, const int* xrp, const int* xci, const double* xv, const int* yrp,
                        const int* yci, const double* yv, const int* crp, int* cci, double* cv, int* overflow);
int spgemm_table_capacity();
// Wide rows (the listed rows; nwg workgroups, each with an ncols-entry slice of mark
// and acc in device memory, mark zeroed before each of the two calls): the same
// canonical order with a dense accumulator, entries written in increasing column.
void launch_spgemm_count_wide(hipStream_t s, int nlist, const int* rows, const int* xrp, const int* xci,
                              const int* yrp, const int* yci, int ncols, int* mark, int nwg, int* counts);
void launch_spgemm_fill_wide(hipStream_t s, int nlist, const int* rows, const int* xrp, const int* xci,
                             const double* xv, const int* yrp, const int* yci, const double* yv, int ncols, int* mark,
                             double* acc, int nwg, const int* crp, int* cci, double* cv, int* overflow);

// Two-point-flux matrix values and log-permeability gradient (tpfa.hip).
void launch_tpfa_values(hipStream_t s, int nx, int ny, int nz, double kz, int dirichlet, const double* logk,
                        const int* rp, double* val);
void launch_tpfa_grad(hipStream_t s, int nx, int ny, int nz, double kz, int dirichlet, const double* logk,
                      const double* lam, const double* x, double* g);

}  // namespace cpc
