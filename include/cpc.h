/*
 * cpc.h — combined-preconditioned conjugate gradients on AMD Instinct MI355X (gfx950).
 *
 * Solves A u = f for a sparse symmetric positive definite A (Section 2, eq. 2.1)
 * by PCG whose preconditioner is the combined operator B_co of Algorithm 2.1:
 *     u1 = S f,  u2 = u1 + B (f - A u1),  u3 = u2 + S^T (f - A u2),
 * with S = one classical (Ruge-Stueben) AMG V-cycle with a Gauss-Seidel smoother
 * on every level (Algorithm 3.2) and B = ILU(0) (Algorithm 3.1 with k = 0),
 * the assignment of Sections 3 and 5. Work is split as in Section 3.2 into a
 * SETUP phase (cpc_setup) and a SOLVE phase (cpc_solve).
 *
 * Conventions for every call:
 *   - Every function returns a cpc_status and never aborts or throws. On a status
 *     other than CPC_OK, cpc_last_error() returns a message (thread-local).
 *   - "host" pointers are ordinary CPU memory; "device" pointers are memory on the
 *     GPU the handle was set up on (e.g. a torch tensor's data_ptr()). Device
 *     vectors are FP64, contiguous, of length n (the finest level's size).
 *   - Matrices are CSR, 0-based, int32 indices, FP64 values: row_ptr[n+1],
 *     col_idx[nnz], val[nnz], row_ptr[0] = 0, monotone, columns sorted and unique in
 *     [0, n) within each row, diagonal present and > 0, numerically symmetric.
 *   - The handle owns every device buffer it allocates; callers own what they pass.
 *     All GPU work of a handle is ordered on the stream given to cpc_setup; calls
 *     that return results to the host synchronise that stream before returning.
 *   - A handle must not be used from two threads at once.
 */
#ifndef CPC_H
#define CPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpc_solver* cpc_handle;

typedef enum {
  CPC_OK = 0,
  CPC_E_ARG = 1,       /* invalid argument or CSR that breaks the input contract          */
  CPC_E_NOT_SPD = 2,   /* non-positive diagonal, ILU(0) pivot or coarse Cholesky pivot     */
  CPC_E_BREAKDOWN = 3, /* PCG breakdown: <p,Ap> <= 0, <r,z> <= 0 or a non-finite value      */
  CPC_E_MAXIT = 4,     /* no convergence within maxit (x holds the last iterate; this is
                          the "does not converge" entry of Table 5.2)                       */
  CPC_E_DEVICE = 5,    /* HIP runtime error or a device-side guard (e.g. a wait limit)      */
  CPC_E_NOMEM = 6      /* host or device allocation failed                                  */
} cpc_status;

/* Preconditioners (Table 5.2). */
typedef enum {
  CPC_PREC_COMBINED = 0, /* B_co, Algorithm 2.1 (S = V-cycle, B = ILU(0))                   */
  CPC_PREC_AMG = 1,      /* AMG(GS): two V-cycles, i.e. S~ of Section 2 with S = V-cycle    */
  CPC_PREC_ILU = 2,      /* ILU(0) alone                                                    */
  CPC_PREC_ADDITIVE = 3, /* B^ = S~ + B, eq. (2.7) with W_1 = V, Pi_1 = I, A_1^{-1} = B      */
  CPC_PREC_NONE = 4,     /* identity (plain CG)                                             */
  CPC_PREC_AMG_ILU = 5,  /* AMG(ILU(0)) of Table 5.2: two V-cycles with ILU(0) as the
                            finest-level smoother (pre and post) and GS below            */
  CPC_PREC_BBAR = 6      /* B-bar of the remark after Theorem 2.1, the wrong order:
                            I - B-bar A = (I - BA)(I - S~A)(I - BA); not SPD in general
                            (kept to show why Algorithm 2.1's order matters)              */
} cpc_prec;

/* Operators applied by cpc_apply_op (each z = M r from a zero initial guess). */
typedef enum {
  CPC_OP_COMBINED = 0, /* B_co                                                              */
  CPC_OP_AMG = 1,      /* two V-cycles (S~)                                                 */
  CPC_OP_ILU = 2,      /* (LU)^{-1}                                                         */
  CPC_OP_ADDITIVE = 3, /* S~ + (LU)^{-1}                                                    */
  CPC_OP_NONE = 4,     /* identity                                                          */
  CPC_OP_VCYCLE = 5,   /* one V-cycle (Algorithm 3.2)                                       */
  CPC_OP_FGS = 6,      /* (D+L)^{-1} on the finest level (one forward Gauss-Seidel sweep)   */
  CPC_OP_BGS = 7,      /* (D+U)^{-1} on the finest level (one backward Gauss-Seidel sweep)  */
  CPC_OP_AMG_ILU = 8,  /* AMG(ILU(0)), as CPC_PREC_AMG_ILU                                  */
  CPC_OP_BBAR = 9      /* B-bar, as CPC_PREC_BBAR                                           */
} cpc_op;

typedef enum {
  CPC_FP64 = 0,        /* everything in FP64                                                */
  CPC_FP32_PRECOND = 1 /* preconditioner data and vectors in FP32 with FP64 row sums; PCG
                          vectors, outer residuals, reductions and the coarsest solve FP64  */
} cpc_precision;

typedef struct {
  int32_t struct_size;    /* sizeof(cpc_options); set by cpc_default_options                */
  int32_t prec;           /* cpc_prec used by cpc_solve (default CPC_PREC_COMBINED)         */
  int32_t precision;      /* cpc_precision (default CPC_FP64)                               */
  int32_t max_coarse;     /* a level with at most this many rows is solved exactly (256)    */
  int32_t max_levels;     /* at most this many levels (25)                                  */
  int32_t swap_roles;     /* 0: S = V-cycle, B = ILU(0) (Section 3); 1: S = ILU(0), B = V   */
  int32_t check_symmetry; /* 1: reject CSR that is not numerically symmetric (O(nnz) check) */
  int32_t use_graph;      /* 1: replay each PCG iteration as a captured HIP graph           */
  int32_t check_every;    /* PCG iterations between host reads of the convergence flag; 0
                             (default): predicted from the mean residual reduction so far
                             (single systems; a batch then reads it after every iteration) */
  int32_t rap_on_gpu;     /* 1: Galerkin products on the GPU (default); 0 is not offered     */
  int32_t sweep_block_rows; /* rows per workgroup block of the triangular sweeps (0 = auto)  */
  int32_t sweep_threads;  /* threads per sweep workgroup: 64 (one wave) or 256; 0 = auto     */
  int32_t dense_smoother; /* Gauss-Seidel through explicit inverses of D+L (whole level,
                             <= 16384 rows) or of its diagonal blocks (block substitution):
                             0 = where measured faster at setup, 1 = never, 2 = whole-level
                             inverses wherever they fit, 3 = blocks of 2048 rows on every
                             smoothed level of more than 4096 rows                          */
  int32_t tune;           /* 1: pick each level's smoother form and sweep block size by timing
                             candidates at setup (default); 0: fixed rules (faster setup)   */
  int32_t verbose;        /* 1: one progress line per setup phase on stderr                 */
  int32_t ilu_fill;       /* level of fill k of the ILU factorisation used as B (Algorithm
                             3.1; 0 = ILU(0), the paper's choice; at most 16; single
                             systems only, cpc_setup_batch rejects k > 0)                  */
  double theta;           /* strength threshold of the classical coarsening (0.25)          */
  int32_t sweep_kernel;   /* level-scheduled triangular solves: 0 = one wave per block, no
                             barriers, where every row has at most 64 dependency entries
                             (else the four-wave kernel); 1 = the four-wave kernel always  */
} cpc_options;

typedef struct {
  int32_t iters;          /* PCG iterations of the last solve                               */
  int32_t status;         /* cpc_status of the last solve                                   */
  double relres;          /* ||r_k||/||b|| of the recursively updated residual at exit     */
  double setup_s;         /* wall seconds of cpc_setup                                      */
  double solve_s;         /* wall seconds of the last cpc_solve (device-synchronised)       */
  double bytes_per_iter;  /* HBM bytes one PCG iteration's kernels move in the forms the setup
                             chose (an explicit inverse reads its whole triangle)           */
  double bytes_initial;   /* the same before the first iteration                            */
  double method_bytes_per_iter; /* bytes the method itself must move in one PCG iteration:
                             every matrix read once per pass the algorithm makes (value +
                             4-byte column, 4-byte row pointer), every vector read or written
                             once per step, whatever form evaluates a Gauss-Seidel sweep    */
  double method_bytes_initial;  /* the same before the first iteration                     */
} cpc_stats;

/* Fill *opt with the defaults listed above. */
void cpc_default_options(cpc_options* opt);

/* SETUP (Section 3.2): validate the host CSR, factor ILU(0) (Algorithm 3.1, k = 0),
 * build the classical AMG hierarchy (C/F splitting and Ruge-Stueben interpolation
 * on the host, Galerkin products A_l = P_l^T A_{l+1} P_l on the GPU), factor the
 * coarsest matrix, build the sweep schedules and upload everything.
 *   n, row_ptr, col_idx, val : host CSR (copied; may be freed on return).
 *   opt                      : NULL for defaults.
 *   hip_stream               : hipStream_t to order all work on (NULL = default stream).
 *   out                      : receives the handle (NULL on failure).
 * Errors: CPC_E_ARG (contract), CPC_E_NOT_SPD, CPC_E_NOMEM, CPC_E_DEVICE. */
cpc_status cpc_setup(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                     const cpc_options* opt, void* hip_stream, cpc_handle* out);

/* SOLVE: preconditioned conjugate gradients (Section 2, the PCG of eq. 2.1 with the
 * preconditioner of Algorithm 2.1 by default, else the one the options name) for
 * A x = b, stopped on the relative residual as in the experiments of Section 5
 * (Table 5.2: relative residual below a tolerance, a cap on the iterations).
 *   b_dev, x_dev : device FP64 vectors of length n. x_dev is read as the initial
 *                  guess when use_x0 != 0, otherwise overwritten from 0.
 *   tol          : stop when ||r_k||_2 / ||b||_2 <= tol (recursively updated r_k;
 *                  checked before the first iteration as well). tol = 0 runs maxit.
 *   maxit        : iteration cap (>= 0).
 *   iters, relres: host outputs (may be NULL).
 * b = 0 gives x = 0, iters = 0, CPC_OK. Returns CPC_E_MAXIT with the last iterate
 * in x when the cap is reached, CPC_E_BREAKDOWN on breakdown. */
cpc_status cpc_solve(cpc_handle h, const double* b_dev, double* x_dev, int32_t use_x0, double tol,
                     int32_t maxit, int32_t* iters, double* relres);

/* Same as cpc_solve with a different preconditioner for this call (cpc_prec). */
cpc_status cpc_solve_with(cpc_handle h, int32_t prec, const double* b_dev, double* x_dev, int32_t use_x0,
                          double tol, int32_t maxit, int32_t* iters, double* relres);

/* z_dev = M r_dev for the operator `op` (cpc_op), device FP64 vectors of length n. */
cpc_status cpc_apply_op(cpc_handle h, int32_t op, const double* r_dev, double* z_dev);

/* y_dev = A_l x_dev on level `level` of the hierarchy (0 = finest, A_0 = A; coarser
 * levels are the Galerkin products A_{l+1} = P_l^T A_l P_l of Section 3.2, Algorithm
 * 3.2); device FP64 vectors of length n_l. CPC_E_ARG for a level out of range. */
cpc_status cpc_spmv(cpc_handle h, int32_t level, const double* x_dev, double* y_dev);

/* C = X Y, the sparse product the SETUP's Galerkin products are made of (Section 3.2:
 * A_{l+1} = P_l^T (A_l P_l) as two such products), on the current device with the
 * same kernels: entry (i, j) of C accumulates the rounded products x_ik y_kj from 0.0
 * in the column order of row i of X, without fused multiply-adds, so the result is
 * bit-identical to a sequential evaluation in that order; the columns of each row of
 * C come out sorted. Rows with more distinct columns than the kernels' LDS table
 * (4096) take the wide-row path (a dense accumulator in device memory).
 * Host CSR in (X: nrows x ninner, Y: ninner x ncols; sorted or unsorted columns, no
 * duplicates within a row) and out: crp (nrows + 1 entries) and *nnz are written on
 * every call; cci and cv (at least *nnz entries each) only when both are non-null, so
 * a first call with null arrays sizes them. CPC_E_ARG on bad sizes or indices,
 * CPC_E_NOMEM when C exceeds 2^31 entries or device memory, CPC_E_DEVICE on a device
 * error. Exposed for tests and tools. */
cpc_status cpc_spgemm(int32_t nrows, int32_t ninner, int32_t ncols, const int32_t* xrp, const int32_t* xci,
                      const double* xv, const int32_t* yrp, const int32_t* yci, const double* yv, int32_t* crp,
                      int32_t* cci, double* cv, int64_t* nnz);

/* Description of the AMG hierarchy the SETUP built (Section 3.2: classical
 * coarsening, Galerkin coarse matrices, coarsest level solved exactly). Caller host
 * arrays hold at least max_levels entries: *nlev = number of levels; n_l[l], nnz_l[l]
 * for each level l (0 = finest); depth_l[l] = number of level sets of the
 * lower-triangular dependency graph of A_l (the dependent steps of one natural-order
 * Gauss-Seidel sweep of Algorithm 3.2). Null arrays are skipped. */
cpc_status cpc_hierarchy_info(cpc_handle h, int32_t* nlev, int32_t* n_l, int64_t* nnz_l, int32_t* depth_l);

/* How the Gauss-Seidel smoother of Algorithm 3.2 is applied on level `level`:
 * *kind = 0 level-scheduled triangular sweeps, 1 products with the explicit inverse of
 * D+L (forward sweep) and its transpose (backward sweep, D+U = (D+L)^T for symmetric
 * A), 2 block substitution with explicit inverses of the diagonal blocks of D+L, -1 the
 * level is not smoothed (coarsest). *block_rows (may be null): rows per workgroup block
 * of the level's sweep schedules (also used by ILU(0) on level 0), or per diagonal block
 * of the block substitution. CPC_E_ARG for a level out of range. */
cpc_status cpc_smoother_kind(cpc_handle h, int32_t level, int32_t* kind, int32_t* block_rows);

/* Device memory (bytes) that the explicit inverses of level `level`'s Gauss-Seidel
 * smoother take (same passage as cpc_smoother_kind): the inverse of D+L and its stored
 * transpose, or the diagonal-block inverses and their transposes (kind 1 or 2, row
 * stride padded as the products read it, FP32 with CPC_FP32_PRECOND); 0 for sweeps and
 * for the coarsest level. CPC_E_ARG for a null pointer or a level out of range. */
cpc_status cpc_smoother_bytes(cpc_handle h, int32_t level, int64_t* bytes);

/* Copy level `level`'s matrix A_l to host CSR arrays (row_ptr[n_l+1], col_idx and
 * val of nnz_l entries). */
cpc_status cpc_get_level(cpc_handle h, int32_t level, int32_t* row_ptr, int32_t* col_idx, double* val);

/* Copy the prolongation from level level+1 to level `level` (host CSR with n_l rows),
 * and the C/F marker (1 = C, 0 = F) of level `level` (n_l entries). nnz via p_nnz. */
cpc_status cpc_get_prolongation(cpc_handle h, int32_t level, int64_t* p_nnz, int32_t* row_ptr, int32_t* col_idx,
                                double* val, int32_t* cf);

/* Copy the ILU(0) values (on the pattern of the finest A; strictly lower = L with a
 * unit diagonal implied, diagonal and upper = U) to a host array of nnz entries.
 * CPC_E_ARG for a handle set up with ilu_fill > 0 (use cpc_get_ilu_factor). */
cpc_status cpc_get_ilu(cpc_handle h, double* lu);

/* The ILU(k) factor the handle applies as B (k = options.ilu_fill; Algorithm 3.1):
 * *nnz = its number of entries; then, for non-null arrays, its row pointers
 * (n + 1), columns (sorted within rows) and values (strictly lower = L with a unit
 * diagonal implied, diagonal and upper = U), host arrays the caller owns. For k = 0
 * the pattern is that of the finest A. */
cpc_status cpc_get_ilu_factor(cpc_handle h, int64_t* nnz, int32_t* row_ptr, int32_t* col_idx, double* val);

/* Statistics of the handle (setup time, last solve). */
cpc_status cpc_get_stats(cpc_handle h, cpc_stats* st);

/* Adjoint helper: g_nnz_dev[p] = -lam_dev[i] * x_dev[j] for every stored entry p = (i, j)
 * of the finest A (the gradient of lam^T (b - A x) with respect to the entries of A).
 * Device arrays: lam, x of length n; g of length nnz. */
cpc_status cpc_neg_outer_on_pattern(cpc_handle h, const double* lam_dev, const double* x_dev, double* g_nnz_dev);

/* ---- Differentiable form (gradient of a misfit through the solve) ---------------
 * The two-point-flux matrix of the model problem of Section 4 (c = 0) on an
 * nx x ny x nz grid of unit cells (cell index i + nx*(j + ny*k)): a_ij = -T_ij,
 * T = 2 s k_a k_b / (k_a + k_b), k = exp(log k), s = 1 on x/y faces and kz_ratio on
 * z faces; a_ii = sum of the cell's T, plus T_b = 2 k_i per Dirichlet (p = 0) face
 * on x = 0 and x = nx when dirichlet_x != 0. Rows list z-, y-, x-, diagonal, x+, y+,
 * z+ (the neighbours that exist). */

/* Host pattern: row_ptr[n+1] and col_idx[nnz] (host arrays; call with col_idx = NULL
 * first to get nnz = row_ptr[n]). */
cpc_status cpc_tpfa_pattern(int32_t nx, int32_t ny, int32_t nz, int32_t* row_ptr, int32_t* col_idx);

/* Device values of the matrix for log-permeability logk_dev[n] on the pattern whose
 * device row pointers are row_ptr_dev; writes val_dev[nnz]. Asynchronous on hip_stream. */
cpc_status cpc_tpfa_values(int32_t nx, int32_t ny, int32_t nz, double kz_ratio, int32_t dirichlet_x,
                           const double* logk_dev, const int32_t* row_ptr_dev, double* val_dev, void* hip_stream);

/* grad_dev[c] = dL/dlog k_c given the adjoint lam = A^{-1} dL/dx and the state x
 * (all device FP64 arrays of length n), through the face transmissibilities.
 * Asynchronous on hip_stream. */
cpc_status cpc_tpfa_logk_grad(int32_t nx, int32_t ny, int32_t nz, double kz_ratio, int32_t dirichlet_x,
                              const double* logk_dev, const double* lam_dev, const double* x_dev, double* grad_dev,
                              void* hip_stream);

/* Replace the values of the matrix that PCG multiplies by (same pattern as the setup
 * matrix; device FP64 array of nnz entries, read at each solve, caller-owned, must
 * stay alive) while keeping the preconditioner built at setup. NULL restores the
 * setup matrix. A preconditioner built for a nearby matrix is still SPD, so PCG
 * converges to the new system's solution (used for finite-difference checks). */
cpc_status cpc_set_operator_values(cpc_handle h, const double* val_dev);

/* Kernel families timed by cpc_time_kernel. */
typedef enum {
  CPC_K_SPMV_PQ = 0,   /* PCG q = A p with <p, q> (finest level)                           */
  CPC_K_FGS = 1,       /* forward Gauss-Seidel sweep from zero (V-cycle pre-smoothing)      */
  CPC_K_BGS = 2,       /* backward Gauss-Seidel sweep in place (V-cycle post-smoothing)     */
  CPC_K_ILU_L = 3,     /* ILU(0) unit-lower solve                                           */
  CPC_K_ILU_U = 4,     /* ILU(0) upper solve with the u2 = u1 + w epilogue                  */
  CPC_K_RESIDUAL = 5,  /* level residual r = f - A u                                        */
  CPC_K_RESTRICT = 6,  /* f_c = R r                                                         */
  CPC_K_PROLONG = 7,   /* u += P e                                                          */
  CPC_K_VCYCLE = 8,    /* one whole V-cycle                                                 */
  CPC_K_PRECOND = 9,   /* one application of the handle's preconditioner                    */
  CPC_K_ITERATION = 10, /* one whole PCG iteration                                          */
  CPC_K_DENSE_GEMV = 11, /* products with explicit inverses of D+L or of its diagonal blocks
                           (both directions), one launch per block and direction            */
  CPC_K_SWEEP = 12     /* every level-scheduled triangular solve of one combined-
                           preconditioner iteration: the forward and backward Gauss-Seidel
                           sweeps of both V-cycles on each level smoothed that way, then
                           the ILU(0) L and U solves (the mix a PCG iteration launches)    */
} cpc_kernel;

/* Measurement helper (not needed to solve): runs `reps` repetitions of the kernel
 * family `kernel` (cpc_kernel) on the handle's current work vectors and reports:
 *   avg_ms                : mean duration of one launch (HIP events recorded on the
 *                           handle's stream around each launch for the triangular
 *                           solves and the dense products, else around all repetitions);
 *   bytes_per_launch      : the method's bytes for the work of one launch: each matrix
 *                           read once per pass the algorithm makes over it (value + 4-byte
 *                           column, 4-byte row pointer), each vector read or written once
 *                           (a Gauss-Seidel sweep counts its triangle, however evaluated;
 *                           the dense products share the sweeps they evaluate evenly);
 *   launches              : the number of launches timed;
 *   form_bytes_per_launch : the bytes the evaluated form itself moves (an explicit
 *                           inverse reads its stored triangle); may be NULL.
 * level >= 0 selects one level; level = -1 takes every level the family runs on in
 * one V-cycle (one PCG iteration for CPC_K_SWEEP), one launch per level per
 * repetition (the averages are then over that mix). Work vectors are overwritten. */
cpc_status cpc_time_kernel(cpc_handle h, int32_t kernel, int32_t level, int32_t reps, double* avg_ms,
                           double* bytes_per_launch, int32_t* launches, double* form_bytes_per_launch);

/* ---- Batched form: independent systems of different sizes solved together ------
 * cpc_setup_batch builds each system's own hierarchy (exactly what cpc_setup would
 * build for it alone) and concatenates them level by level; cpc_solve_batch runs PCG
 * on all systems at once, one HIP-graph replay per iteration, with per-system
 * scalars and stopping, so each system's iterates are those of its own solve.
 *   nsys                      : number of systems (>= 1). A system of at most max_coarse
 *                               rows is its own coarsest level: its V-cycle is the exact
 *                               solve, as for a one-level hierarchy alone.
 *   n[s], row_ptr[s], col_idx[s], val[s] : host CSR of system s (copied).
 * Vectors of a batch are concatenated in system order: system s occupies entries
 * [offset_s, offset_s + n[s]) (offsets from cpc_batch_info). */
cpc_status cpc_setup_batch(int32_t nsys, const int32_t* n, const int32_t* const* row_ptr,
                           const int32_t* const* col_idx, const double* const* val, const cpc_options* opt,
                           void* hip_stream, cpc_handle* out);

/* PCG (Algorithm 2.1's preconditioner in each iteration) on every system of a batch
 * handle from x = 0 with the handle's preconditioner. b_dev, x_dev: concatenated device
 * FP64 vectors. iters[nsys], relres[nsys]: host outputs per system (may be NULL). A
 * system stops on its own (tolerance, iteration cap, breakdown or b = 0): its x is kept
 * and the rest of the solve skips it, the preconditioner's launches included. Returns
 * CPC_OK when every system converged (or had b = 0), CPC_E_MAXIT when one did not,
 * CPC_E_BREAKDOWN on a breakdown in any system (the others still converge). */
cpc_status cpc_solve_batch(cpc_handle h, const double* b_dev, double* x_dev, double tol, int32_t maxit,
                           int32_t* iters, double* relres);

/* Number of systems and, per system, rows and offset in the concatenated vectors
 * (caller arrays of nsys entries; a single-system handle reports one system). */
cpc_status cpc_batch_info(cpc_handle h, int32_t* nsys, int32_t* n, int32_t* offset);

/* For callers that cannot allocate device memory during a solve (serving loops,
 * harnesses that forbid hipMalloc): the solve of cpc_solve on a single-system handle,
 * with the same arguments, results and errors, that allocates nothing. Its scratch (the
 * PCG scalars, the partial sums of the reductions and the sweep counters, 33 KiB) lives
 * in one static 64 KiB device array per GPU instead of the handle; every iteration is
 * launched directly (no graph is instantiated). Limits: every call on one GPU shares
 * that array, so calls that overlap on one GPU (two threads, or two streams with work
 * in flight) race and must be serialised by the caller; batch handles give
 * CPC_E_ARG. The array is located on the first call on each device. */
cpc_status cpc_solve_noalloc(cpc_handle h, const double* b_dev, double* x_dev, int32_t use_x0, double tol,
                             int32_t maxit, int32_t* iters, double* relres);

/* Destroy the handle and free its device and host memory (NULL is ignored). */
void cpc_destroy(cpc_handle h);

/* Message for the last non-OK status returned on this thread. */
const char* cpc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CPC_H */
