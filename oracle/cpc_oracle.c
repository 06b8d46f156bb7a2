/*
 * Oracle for the combined-preconditioned conjugate gradient method of
 * "Combined Preconditioning with Applications in Reservoir Simulation"
 * (Hu, Wu, Wu, Xu, Zhang, Zhang, Zikatanov).
 *
 * TEST INFRASTRUCTURE ONLY. This file is a plain, slow, sequential FP64
 * reference used by the tests, by the smoke check and by the CPU-baseline leg
 * of the benchmark. The product library never links, loads or calls it, and
 * it shares no code with the product.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -o liboracle.so cpc_oracle.c -lm
 * (no FMA contraction: every a*b+c is a rounded product then a rounded sum).
 *
 * What it computes, in the paper's order and notation:
 *   - ILU(0): Algorithm 3.1 with k = 0 (level of fill 0 keeps exactly the
 *     pattern of A), in the IKJ form the paper takes from Saad.
 *   - AMG SETUP (Section 3.2): classical Ruge-Stueben C/F splitting and classical
 *     interpolation P_l, Galerkin A_l = P_l^T A_{l+1} P_l, exact solve on the
 *     coarsest level (dense Cholesky).
 *   - V-cycle (Algorithm 3.2) with one forward Gauss-Seidel sweep as S_l and its
 *     adjoint, one backward sweep, as S_l^T (Section 3.3).
 *   - Combined preconditioner (Algorithm 2.1): S = one V-cycle, B = ILU(0)
 *     (the assignment of Section 3 and of the experiments in Section 5).
 *   - Comparators of Table 5.2: ILU(0) alone, AMG(GS) with two cycles, AMG(ILU(0))
 *     (ILU(0) as the finest-level smoother, GS below, two cycles), and the
 *     additive form S~ + B of eq. (2.7) with W_1 = V, A_1^{-1} = B.
 *   - The wrong-order composition B-bar of the remark after Theorem 2.1, which is
 *     not SPD in general (the negative case the remark warns about).
 *   - PCG stopped on the relative residual of the recursively updated residual.
 *
 * Readings where the paper is silent (strength threshold, tie-breaks, second
 * pass, interpolation formula, coarsest-level rule) are stated at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_E_ARG = 1, OR_E_NOT_SPD = 2, OR_E_BREAKDOWN = 3, OR_E_MAXIT = 4, OR_E_NOMEM = 6 };

/* preconditioner selectors for or_apply / or_pcg */
enum {
  OR_PREC_COMBINED = 0, /* B_co, Algorithm 2.1, S = V-cycle, B = ILU(0)            */
  OR_PREC_AMG = 1,      /* AMG(GS): two V-cycles = S~ with S = V-cycle            */
  OR_PREC_ILU = 2,      /* ILU(0) alone                                           */
  OR_PREC_ADDITIVE = 3, /* B^ = S~ + B, eq. (2.7)                                 */
  OR_PREC_NONE = 4,     /* identity                                               */
  OR_OP_VCYCLE = 5,     /* one V-cycle from zero                                  */
  OR_OP_FGS = 6,        /* forward GS from zero on the finest level, (D+L)^{-1}   */
  OR_OP_BGS = 7,        /* backward GS from zero on the finest level, (D+U)^{-1}  */
  OR_OP_COMBINED_GS = 8,/* Algorithm 2.1 with S = (D+L)^{-1}, S^T = (D+U)^{-1}, B = ILU(0) */
  OR_OP_COMBINED_SWAP = 9, /* Algorithm 2.1 with S = ILU(0), B = V-cycle          */
  OR_PREC_AMG_ILU = 10, /* AMG(ILU(0)) of Table 5.2: two V-cycles whose finest-level
                           smoother is ILU(0) (GS below)                          */
  OR_PREC_BBAR = 11     /* the wrong-order B-bar of Remark 2.1:
                           I - B-bar A = (I - BA)(I - S~A)(I - BA)               */
};

#define OR_MAXLEV 64

typedef struct {
  int n;
  int *rp, *ci;
  double *v;
} or_csr;

typedef struct {
  double theta;
  int max_coarse;
  int max_levels;
  int check_symmetry;
  double s_scale; /* S := s_scale * S inside Algorithm 2.1 (1 = the method; 0 = degenerate S = 0) */
  double b_scale; /* B := b_scale * B inside Algorithm 2.1 and eq. (2.7) (Theorem 2.2 scales B) */
  int ilu_k;      /* level of fill of the ILU factorisation B (Algorithm 3.1); 0 = ILU(0) */
} or_opts;

typedef struct {
  /* depth d = 0 is the finest level; in the paper's numbering it is l = L - d */
  int nlev;
  or_csr A[OR_MAXLEV];
  or_csr P[OR_MAXLEV]; /* P[d]: level d+1 (coarse) -> level d (fine), i.e. P_{L-d-1} */
  or_csr R[OR_MAXLEV]; /* R[d] = P[d]^T stored explicitly                          */
  int *cf[OR_MAXLEV];  /* C/F marker of level d: 1 = C, 0 = F (levels that were split) */
  int n0;              /* coarsest size                                                  */
  double *chol;        /* lower Cholesky factor of the coarsest matrix, row-major n0 x n0 */
  double *lu;          /* ILU(0) values on the pattern of the finest A                   */
  or_csr F;            /* the ILU(k) factor applied as B: L strictly lower (unit diagonal
                          implied), U on and above the diagonal; for k = 0 the pattern of A */
  int *flev;           /* level of fill of every entry of F                              */
  double *work;        /* scratch vectors                                                 */
  double s_scale, b_scale;
} or_hier;

static void csr_free(or_csr* a) {
  free(a->rp);
  free(a->ci);
  free(a->v);
  a->rp = a->ci = NULL;
  a->v = NULL;
}

static int csr_alloc(or_csr* a, int n, long nnz) {
  a->n = n;
  a->rp = (int*)calloc((size_t)n + 1, sizeof(int));
  a->ci = (int*)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
  a->v = (double*)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  return (a->rp && a->ci && a->v) ? OR_OK : OR_E_NOMEM;
}

/* position of column j in row i, or -1 (binary search: columns are sorted) */
static long csr_find(const or_csr* a, int i, int j) {
  long lo = a->rp[i], hi = (long)a->rp[i + 1] - 1;
  while (lo <= hi) {
    long mid = (lo + hi) / 2;
    if (a->ci[mid] == j) return mid;
    if (a->ci[mid] < j) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* ------------------------------------------------------------------ */
/* Input contract: square CSR, sorted unique columns, positive diagonal,
 * numerically symmetric (when asked). */
int or_validate(int n, const int* rp, const int* ci, const double* v, int check_symmetry) {
  if (n <= 0 || !rp || !ci || !v) return OR_E_ARG;
  if (rp[0] != 0) return OR_E_ARG;
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return OR_E_ARG;
    int has_diag = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      if (ci[p] < 0 || ci[p] >= n) return OR_E_ARG;
      if (p > rp[i] && ci[p] <= ci[p - 1]) return OR_E_ARG;
      if (!isfinite(v[p])) return OR_E_ARG;
      if (ci[p] == i) {
        has_diag = 1;
        if (!(v[p] > 0.0)) return OR_E_NOT_SPD;
      }
    }
    if (!has_diag) return OR_E_ARG;
  }
  if (check_symmetry) {
    or_csr a = {n, (int*)rp, (int*)ci, (double*)v};
    for (int i = 0; i < n; ++i)
      for (int p = rp[i]; p < rp[i + 1]; ++p) {
        long q = csr_find(&a, ci[p], i);
        if (q < 0) return OR_E_ARG;
        double x = v[p], y = v[q];
        if (fabs(x - y) > 1e-12 * fmax(fabs(x), fabs(y))) return OR_E_ARG;
      }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* ILU(0), Algorithm 3.1 with k = 0. Row i is eliminated with every earlier row
 * m that it is coupled to (increasing m): a_im := a_im / a_mm, then
 * a_ij := a_ij - a_im a_mj for the j > m that lie in the pattern of row i.
 * Entries outside the pattern have level of fill >= 1 and are dropped.
 * Result: lu[] on the pattern of A; strictly lower part = L (unit diagonal
 * implied), diagonal and upper part = U. Returns OR_E_NOT_SPD on a pivot <= 0. */
int or_ilu0(int n, const int* rp, const int* ci, const double* v, double* lu) {
  memcpy(lu, v, sizeof(double) * (size_t)rp[n]);
  long* pos = (long*)malloc(sizeof(long) * (size_t)n);
  long* diag = (long*)malloc(sizeof(long) * (size_t)n);
  if (!pos || !diag) { free(pos); free(diag); return OR_E_NOMEM; }
  for (int j = 0; j < n; ++j) pos[j] = -1;
  int status = OR_OK;
  for (int i = 0; i < n && status == OR_OK; ++i) {
    diag[i] = -1;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      pos[ci[p]] = p;
      if (ci[p] == i) diag[i] = p;
    }
    for (int p = rp[i]; p < rp[i + 1] && ci[p] < i; ++p) {
      int m = ci[p];
      lu[p] = lu[p] / lu[diag[m]];
      for (int q = diag[m] + 1; q < rp[m + 1]; ++q) {
        long t = pos[ci[q]];
        if (t >= 0) lu[t] = lu[t] - lu[p] * lu[q];
      }
    }
    if (!(lu[diag[i]] > 0.0)) status = OR_E_NOT_SPD;
    for (int p = rp[i]; p < rp[i + 1]; ++p) pos[ci[p]] = -1;
  }
  free(pos);
  free(diag);
  return status;
}

/* ------------------------------------------------------------------ */
/* ILU(k), Algorithm 3.1 with the level of fill of its definition. Row i starts as
 * row i of A with level 0 on its entries (the diagonal included). For m < i in
 * increasing order, if the current level of (i, m) is at most k:
 *   a_im := a_im / u_mm, then for every stored entry (m, j), j > m, of the factor:
 *   a_ij := a_ij - a_im u_mj (an entry not yet in row i enters as 0 first) and
 *   lev_ij := min(lev_ij, lev_im + lev_mj + 1).
 * Entries created in row i join the sweep over m in column order. At the end of
 * the row every entry with level above k is dropped. Output (malloc'ed, freed with
 * or_free_buf): frp[n+1], fci/fv/flev[nnz] sorted by column. For k = 0 the
 * pattern is that of A and the values are those of or_ilu0. */
#define OR_LEV_INF (1 << 28)
int or_iluk(int n, const int* rp, const int* ci, const double* v, int k, int** frp_out, int** fci_out,
            double** fv_out, int** flev_out) {
  int* frp = (int*)malloc(sizeof(int) * ((size_t)n + 1));
  int* fdiag = (int*)malloc(sizeof(int) * (size_t)n);
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  int* lv = (int*)malloc(sizeof(int) * (size_t)n);
  int* nxt = (int*)malloc(sizeof(int) * ((size_t)n + 1));
  long cap = (long)rp[n] + n + 16, nnz = 0;
  int* fci = (int*)malloc(sizeof(int) * (size_t)cap);
  double* fv = (double*)malloc(sizeof(double) * (size_t)cap);
  int* flev = (int*)malloc(sizeof(int) * (size_t)cap);
  int status = OR_OK;
  if (!frp || !fdiag || !w || !lv || !nxt || !fci || !fv || !flev) { status = OR_E_NOMEM; goto out; }
  for (int j = 0; j < n; ++j) lv[j] = -1; /* -1: column not in the working row */
  frp[0] = 0;
  for (int i = 0; i < n && status == OR_OK; ++i) {
    /* working row: a sorted linked list of columns, head at index n */
    int last = n;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      w[j] = v[p];
      lv[j] = 0;
      nxt[last] = j;
      last = j;
    }
    nxt[last] = -1;
    for (int m = nxt[n]; m >= 0 && m < i; m = nxt[m]) {
      if (lv[m] > k) continue;
      w[m] = w[m] / fv[fdiag[m]];
      int at = m; /* insertion point: the list is sorted and every j below is > m */
      for (int q = fdiag[m] + 1; q < frp[m + 1]; ++q) {
        int j = fci[q];
        if (lv[j] < 0) {
          while (nxt[at] >= 0 && nxt[at] < j) at = nxt[at];
          nxt[j] = nxt[at];
          nxt[at] = j;
          w[j] = 0.0;
          lv[j] = OR_LEV_INF;
        }
        w[j] = w[j] - w[m] * fv[q];
        int l = lv[m] + flev[q] + 1;
        if (l < lv[j]) lv[j] = l;
        at = j;
      }
    }
    /* keep the entries of level <= k */
    for (int j = nxt[n]; j >= 0; j = nxt[j]) {
      if (lv[j] <= k) {
        if (nnz == cap) {
          cap = 2 * cap;
          int* a = (int*)realloc(fci, sizeof(int) * (size_t)cap);
          if (a) fci = a;
          double* b = (double*)realloc(fv, sizeof(double) * (size_t)cap);
          if (b) fv = b;
          int* c = (int*)realloc(flev, sizeof(int) * (size_t)cap);
          if (c) flev = c;
          if (!a || !b || !c) { status = OR_E_NOMEM; break; }
        }
        if (j == i) fdiag[i] = (int)nnz;
        fci[nnz] = j;
        fv[nnz] = w[j];
        flev[nnz] = lv[j];
        nnz++;
      }
    }
    for (int j = nxt[n]; j >= 0; j = nxt[j]) lv[j] = -1;
    frp[i + 1] = (int)nnz;
    if (status == OR_OK && !(fv[fdiag[i]] > 0.0)) status = OR_E_NOT_SPD;
  }
out:
  free(fdiag);
  free(w);
  free(lv);
  free(nxt);
  if (status != OR_OK) {
    free(frp);
    free(fci);
    free(fv);
    free(flev);
    return status;
  }
  *frp_out = frp;
  *fci_out = fci;
  *fv_out = fv;
  *flev_out = flev;
  return OR_OK;
}

void or_free_buf(void* p) { free(p); }

/* ------------------------------------------------------------------ */
/* Classical Ruge-Stueben coarsening of one level.
 * Strength: j is a strong coupling of i (j in S_i) iff j != i, a_ij < 0 and
 *   -a_ij >= theta * max_{k != i} (-a_ik). Positive couplings are weak.
 * First pass: points with S_i empty become F. lambda_i = |S_i^T intersect U|
 *   (U = undecided). Repeatedly the undecided point with the largest lambda
 *   (ties: smallest index) becomes C; every undecided j in S_i^T becomes F and,
 *   for each such j, every undecided k in S_j gets lambda_k += 1; then every
 *   undecided j in S_i gets lambda_j -= 1.
 * Second pass, F points in increasing index: C_i = S_i intersect C; for each
 *   F point j in S_i (increasing) with no strong coupling into C_i: if a
 *   tentative point already exists, i becomes C and its processing stops;
 *   otherwise j becomes tentative and joins C_i. A surviving tentative point
 *   becomes C.
 * cf[i] = 1 for C, 0 for F. Returns the number of C points. */

typedef struct { int lam; int idx; } heap_item;

static int heap_less(heap_item a, heap_item b) { /* a has priority over b */
  if (a.lam != b.lam) return a.lam > b.lam;
  return a.idx < b.idx;
}

static void heap_push(heap_item* h, long* sz, heap_item x) {
  long c = (*sz)++;
  h[c] = x;
  while (c > 0) {
    long p = (c - 1) / 2;
    if (!heap_less(h[c], h[p])) break;
    heap_item t = h[c]; h[c] = h[p]; h[p] = t;
    c = p;
  }
}

static heap_item heap_pop(heap_item* h, long* sz) {
  heap_item top = h[0];
  h[0] = h[--(*sz)];
  long c = 0;
  for (;;) {
    long l = 2 * c + 1, r = l + 1, best = c;
    if (l < *sz && heap_less(h[l], h[best])) best = l;
    if (r < *sz && heap_less(h[r], h[best])) best = r;
    if (best == c) break;
    heap_item t = h[c]; h[c] = h[best]; h[best] = t;
    c = best;
  }
  return top;
}

/* strength graph S (CSR, same row order) and its transpose ST */
static int strength(const or_csr* a, double theta, or_csr* S, or_csr* ST) {
  int n = a->n;
  long nnz = a->rp[n];
  if (csr_alloc(S, n, nnz) || csr_alloc(ST, n, nnz)) return OR_E_NOMEM;
  long cnt = 0;
  S->rp[0] = 0;
  for (int i = 0; i < n; ++i) {
    double mx = 0.0;
    int any = 0;
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p)
      if (a->ci[p] != i) {
        double t = -a->v[p];
        if (!any || t > mx) mx = t;
        any = 1;
      }
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
      int j = a->ci[p];
      if (j != i && a->v[p] < 0.0 && -a->v[p] >= theta * mx) S->ci[cnt++] = j;
    }
    S->rp[i + 1] = (int)cnt;
  }
  /* transpose */
  for (int i = 0; i <= n; ++i) ST->rp[i] = 0;
  for (long p = 0; p < cnt; ++p) ST->rp[S->ci[p] + 1]++;
  for (int i = 0; i < n; ++i) ST->rp[i + 1] += ST->rp[i];
  int* fill = (int*)malloc(sizeof(int) * (size_t)n);
  if (!fill) return OR_E_NOMEM;
  for (int i = 0; i < n; ++i) fill[i] = ST->rp[i];
  for (int i = 0; i < n; ++i)
    for (int p = S->rp[i]; p < S->rp[i + 1]; ++p) ST->ci[fill[S->ci[p]]++] = i; /* rows ascending */
  free(fill);
  return OR_OK;
}

static int rs_split(const or_csr* a, double theta, int* cf) {
  int n = a->n;
  or_csr S = {0}, ST = {0};
  int st = strength(a, theta, &S, &ST);
  if (st) { csr_free(&S); csr_free(&ST); return -1; }
  enum { UND = -1, FPT = 0, CPT = 1 };
  int* lam = (int*)malloc(sizeof(int) * (size_t)n);
  long heap_cap = (long)n + 4L * (long)S.rp[n] + 16;
  heap_item* heap = (heap_item*)malloc(sizeof(heap_item) * (size_t)heap_cap);
  if (!lam || !heap) { free(lam); free(heap); csr_free(&S); csr_free(&ST); return -1; }
  long hsz = 0;
  for (int i = 0; i < n; ++i) cf[i] = UND;
  for (int i = 0; i < n; ++i)
    if (S.rp[i + 1] == S.rp[i]) cf[i] = FPT; /* no strong couplings: F, empty P row */
  for (int i = 0; i < n; ++i) {
    if (cf[i] != UND) continue;
    int c = 0;
    for (int p = ST.rp[i]; p < ST.rp[i + 1]; ++p)
      if (cf[ST.ci[p]] == UND) c++;
    lam[i] = c;
    heap_item it = {c, i};
    heap_push(heap, &hsz, it);
  }
  /* lazy heap: an entry is current iff the point is undecided and its lam matches */
  while (hsz > 0) {
    heap_item top = heap_pop(heap, &hsz);
    int i = top.idx;
    if (cf[i] != UND || lam[i] != top.lam) continue;
    cf[i] = CPT;
    for (int p = ST.rp[i]; p < ST.rp[i + 1]; ++p) {
      int j = ST.ci[p];
      if (cf[j] != UND) continue;
      cf[j] = FPT;
      for (int q = S.rp[j]; q < S.rp[j + 1]; ++q) {
        int k = S.ci[q];
        if (cf[k] == UND) {
          lam[k] += 1;
          if (hsz >= heap_cap) goto oom;
          heap_item it = {lam[k], k};
          heap_push(heap, &hsz, it);
        }
      }
    }
    for (int p = S.rp[i]; p < S.rp[i + 1]; ++p) {
      int j = S.ci[p];
      if (cf[j] == UND) {
        lam[j] -= 1;
        if (hsz >= heap_cap) goto oom;
        heap_item it = {lam[j], j};
        heap_push(heap, &hsz, it);
      }
    }
  }
  free(heap);
  heap = NULL;

  /* second pass */
  {
    int* mark = (int*)malloc(sizeof(int) * (size_t)n); /* mark[k] == i+1 : k in C_i */
    if (!mark) goto oom;
    for (int k = 0; k < n; ++k) mark[k] = 0;
    for (int i = 0; i < n; ++i) {
      if (cf[i] != FPT) continue;
      int tag = i + 1;
      for (int p = S.rp[i]; p < S.rp[i + 1]; ++p)
        if (cf[S.ci[p]] == CPT) mark[S.ci[p]] = tag;
      int tentative = -1;
      int i_became_c = 0;
      for (int p = S.rp[i]; p < S.rp[i + 1]; ++p) {
        int j = S.ci[p];
        if (cf[j] != FPT) continue;
        int shares = 0;
        for (int q = S.rp[j]; q < S.rp[j + 1]; ++q)
          if (mark[S.ci[q]] == tag) { shares = 1; break; }
        if (shares) continue;
        if (tentative >= 0) {
          cf[i] = CPT;
          i_became_c = 1;
          break;
        }
        tentative = j;
        mark[j] = tag;
      }
      if (!i_became_c && tentative >= 0) cf[tentative] = CPT;
    }
    free(mark);
  }
  free(lam);
  csr_free(&S);
  csr_free(&ST);
  {
    int nc = 0;
    for (int i = 0; i < n; ++i) nc += (cf[i] == CPT);
    return nc;
  }
oom:
  free(heap);
  free(lam);
  csr_free(&S);
  csr_free(&ST);
  return -1;
}

/* ------------------------------------------------------------------ */
/* Classical Ruge-Stueben interpolation for the splitting cf.
 * C point i: unit row to its coarse index (rank among C points in fine order).
 * F point i with strong set S_i: C_i = S_i intersect C, D^s_i = S_i intersect F,
 * D^w_i = the remaining off-diagonals (weak couplings of either sign, and weak
 * or strong C points outside S_i... i.e. everything not in C_i or D^s_i).
 * With abar_mk = a_mk when its sign is opposite to a_mm (else 0),
 *   w_ij = -( a_ij + sum_{m in D^s_i} a_im abar_mj / sum_{k in C_i} abar_mk )
 *           / ( a_ii + sum_{n in D^w_i} a_in ),   j in C_i.
 * A strong F point m with sum_{k in C_i} abar_mk = 0 is moved to D^w_i.
 * Evaluation order (fixed): the denominator sums over row i in increasing column;
 * each numerator starts from a_ij and adds the m terms in increasing m, each term
 * computed as (a_im * abar_mj) / den_m; den_m sums row m in increasing column.
 * S_i empty: empty row. No truncation. */
static int rs_interp(const or_csr* a, double theta, const int* cf, or_csr* P) {
  int n = a->n;
  or_csr S = {0}, ST = {0};
  if (strength(a, theta, &S, &ST)) { csr_free(&S); csr_free(&ST); return OR_E_NOMEM; }
  int* cidx = (int*)malloc(sizeof(int) * (size_t)n);
  int* mark = (int*)malloc(sizeof(int) * (size_t)n); /* 1: in C_i, 2: in D^s_i (strong F) */
  double* num = (double*)malloc(sizeof(double) * (size_t)n);
  if (!cidx || !mark || !num) { free(cidx); free(mark); free(num); csr_free(&S); csr_free(&ST); return OR_E_NOMEM; }
  int nc = 0;
  long nnzP = 0;
  for (int i = 0; i < n; ++i) {
    cidx[i] = cf[i] ? nc++ : -1;
    mark[i] = 0;
  }
  /* count */
  for (int i = 0; i < n; ++i) {
    if (cf[i]) { nnzP += 1; continue; }
    for (int p = S.rp[i]; p < S.rp[i + 1]; ++p) if (cf[S.ci[p]]) nnzP++;
  }
  if (csr_alloc(P, n, nnzP)) { free(cidx); free(mark); free(num); csr_free(&S); csr_free(&ST); return OR_E_NOMEM; }
  long w = 0;
  P->rp[0] = 0;
  for (int i = 0; i < n; ++i) {
    if (cf[i]) {
      P->ci[w] = cidx[i];
      P->v[w] = 1.0;
      w++;
      P->rp[i + 1] = (int)w;
      continue;
    }
    /* classify the strong couplings of i */
    for (int p = S.rp[i]; p < S.rp[i + 1]; ++p) mark[S.ci[p]] = cf[S.ci[p]] ? 1 : 2;
    /* strong F points whose sum over C_i of abar vanishes move to D^w */
    for (int p = S.rp[i]; p < S.rp[i + 1]; ++p) {
      int m = S.ci[p];
      if (mark[m] != 2) continue;
      double amm = 0.0;
      for (int q = a->rp[m]; q < a->rp[m + 1]; ++q) if (a->ci[q] == m) amm = a->v[q];
      double den = 0.0;
      for (int q = a->rp[m]; q < a->rp[m + 1]; ++q) {
        int k = a->ci[q];
        if (k != m && mark[k] == 1 && (a->v[q] < 0.0) != (amm < 0.0)) den = den + a->v[q];
      }
      if (den == 0.0) mark[m] = 3; /* moved to D^w */
    }
    /* denominator a_ii + sum over D^w */
    double aii = 0.0, dsum = 0.0;
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) if (a->ci[p] == i) aii = a->v[p];
    dsum = aii;
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
      int j = a->ci[p];
      if (j == i) continue;
      if (mark[j] == 1 || mark[j] == 2) continue;
      dsum = dsum + a->v[p];
    }
    /* numerators start from a_ij for j in C_i */
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
      int j = a->ci[p];
      if (mark[j] == 1) num[j] = a->v[p];
    }
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
      int m = a->ci[p];
      if (mark[m] != 2) continue;
      double aim = a->v[p];
      double amm = 0.0;
      for (int q = a->rp[m]; q < a->rp[m + 1]; ++q) if (a->ci[q] == m) amm = a->v[q];
      double den = 0.0;
      for (int q = a->rp[m]; q < a->rp[m + 1]; ++q) {
        int k = a->ci[q];
        if (k != m && mark[k] == 1 && (a->v[q] < 0.0) != (amm < 0.0)) den = den + a->v[q];
      }
      for (int q = a->rp[m]; q < a->rp[m + 1]; ++q) {
        int j = a->ci[q];
        if (j != m && mark[j] == 1 && (a->v[q] < 0.0) != (amm < 0.0)) {
          double t = aim * a->v[q];
          t = t / den;
          num[j] = num[j] + t;
        }
      }
    }
    for (int p = S.rp[i]; p < S.rp[i + 1]; ++p) {
      int j = S.ci[p];
      if (mark[j] == 1) {
        P->ci[w] = cidx[j];
        P->v[w] = -(num[j] / dsum);
        w++;
      }
    }
    P->rp[i + 1] = (int)w;
    for (int p = S.rp[i]; p < S.rp[i + 1]; ++p) mark[S.ci[p]] = 0;
  }
  free(cidx);
  free(mark);
  free(num);
  csr_free(&S);
  csr_free(&ST);
  return OR_OK;
}

static int csr_transpose(const or_csr* a, int ncols, or_csr* t) {
  long nnz = a->rp[a->n];
  if (csr_alloc(t, ncols, nnz)) return OR_E_NOMEM;
  for (int j = 0; j <= ncols; ++j) t->rp[j] = 0;
  for (long p = 0; p < nnz; ++p) t->rp[a->ci[p] + 1]++;
  for (int j = 0; j < ncols; ++j) t->rp[j + 1] += t->rp[j];
  int* fill = (int*)malloc(sizeof(int) * (size_t)(ncols > 0 ? ncols : 1));
  if (!fill) return OR_E_NOMEM;
  for (int j = 0; j < ncols; ++j) fill[j] = t->rp[j];
  for (int i = 0; i < a->n; ++i)
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
      long q = fill[a->ci[p]]++;
      t->ci[q] = i;
      t->v[q] = a->v[p];
    }
  free(fill);
  return OR_OK;
}

/* C = X * Y (rows of X times Y), ncols = number of columns of Y. Each entry is
 * accumulated from 0.0 in increasing order of the inner index (the column order
 * of the row of X), products rounded before the add. The pattern is the full
 * symbolic product (no dropping); columns sorted. */
static int csr_matmul(const or_csr* X, const or_csr* Y, int ncols, or_csr* C) {
  int n = X->n;
  int* mark = (int*)malloc(sizeof(int) * (size_t)(ncols > 0 ? ncols : 1));
  double* acc = (double*)malloc(sizeof(double) * (size_t)(ncols > 0 ? ncols : 1));
  int* cols = (int*)malloc(sizeof(int) * (size_t)(ncols > 0 ? ncols : 1));
  if (!mark || !acc || !cols) { free(mark); free(acc); free(cols); return OR_E_NOMEM; }
  for (int j = 0; j < ncols; ++j) mark[j] = -1;
  /* symbolic count */
  long nnz = 0;
  for (int i = 0; i < n; ++i) {
    for (int p = X->rp[i]; p < X->rp[i + 1]; ++p) {
      int k = X->ci[p];
      for (int q = Y->rp[k]; q < Y->rp[k + 1]; ++q)
        if (mark[Y->ci[q]] != i) { mark[Y->ci[q]] = i; nnz++; }
    }
  }
  if (nnz > 2147483647L || csr_alloc(C, n, nnz)) { free(mark); free(acc); free(cols); return OR_E_NOMEM; }
  for (int j = 0; j < ncols; ++j) mark[j] = -1;
  long w = 0;
  C->rp[0] = 0;
  for (int i = 0; i < n; ++i) {
    int nc = 0;
    for (int p = X->rp[i]; p < X->rp[i + 1]; ++p) {
      int k = X->ci[p];
      double xik = X->v[p];
      for (int q = Y->rp[k]; q < Y->rp[k + 1]; ++q) {
        int j = Y->ci[q];
        if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; cols[nc++] = j; }
        double prod = xik * Y->v[q];
        acc[j] = acc[j] + prod;
      }
    }
    /* sort the row's columns (insertion sort: rows are short) */
    for (int s = 1; s < nc; ++s) {
      int c = cols[s], t = s - 1;
      while (t >= 0 && cols[t] > c) { cols[t + 1] = cols[t]; t--; }
      cols[t + 1] = c;
    }
    for (int s = 0; s < nc; ++s) { C->ci[w] = cols[s]; C->v[w] = acc[cols[s]]; w++; }
    C->rp[i + 1] = (int)w;
  }
  free(mark);
  free(acc);
  free(cols);
  return OR_OK;
}

/* Galerkin coarse matrix A_c = P^T A P, formed as R (A P) with R = P^T. */
static int galerkin(const or_csr* A, const or_csr* P, const or_csr* R, int nc, or_csr* Ac) {
  or_csr AP = {0};
  int st = csr_matmul(A, P, nc, &AP);
  if (st) { csr_free(&AP); return st; }
  st = csr_matmul(R, &AP, nc, Ac);
  csr_free(&AP);
  return st;
}

/* dense Cholesky A = G G^T, G lower, row-major; OR_E_NOT_SPD if not positive definite */
static int dense_cholesky(const or_csr* a, double* g) {
  int n = a->n;
  for (long t = 0; t < (long)n * n; ++t) g[t] = 0.0;
  for (int i = 0; i < n; ++i)
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) g[(long)i * n + a->ci[p]] = a->v[p];
  for (int j = 0; j < n; ++j) {
    double d = g[(long)j * n + j];
    for (int k = 0; k < j; ++k) d = d - g[(long)j * n + k] * g[(long)j * n + k];
    if (!(d > 0.0)) return OR_E_NOT_SPD;
    d = sqrt(d);
    g[(long)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = g[(long)i * n + j];
      for (int k = 0; k < j; ++k) s = s - g[(long)i * n + k] * g[(long)j * n + k];
      g[(long)i * n + j] = s / d;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) g[(long)i * n + j] = 0.0;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
void or_default_opts(or_opts* o) {
  o->theta = 0.25;
  o->max_coarse = 256;
  o->max_levels = 25;
  o->check_symmetry = 1;
  o->s_scale = 1.0;
  o->b_scale = 1.0;
  o->ilu_k = 0;
}

void or_free(or_hier* h) {
  if (!h) return;
  for (int d = 0; d < OR_MAXLEV; ++d) {
    csr_free(&h->A[d]);
    csr_free(&h->P[d]);
    csr_free(&h->R[d]);
    free(h->cf[d]);
  }
  free(h->chol);
  free(h->lu);
  csr_free(&h->F);
  free(h->flev);
  free(h->work);
  free(h);
}

/* SETUP phase: ILU(0) of the finest matrix, then the AMG hierarchy.
 * Coarsening stops at a level with n <= max_coarse, at level max_levels, or when
 * the splitting stalls (n_c = 0 or n_c > 0.9 n); that level is solved exactly. */
or_hier* or_setup(int n, const int* rp, const int* ci, const double* v, const or_opts* opt, int* status) {
  or_opts o;
  if (opt) o = *opt; else or_default_opts(&o);
  *status = or_validate(n, rp, ci, v, o.check_symmetry);
  if (*status) return NULL;
  if (o.max_levels < 1) o.max_levels = 1;
  if (o.max_levels > OR_MAXLEV) o.max_levels = OR_MAXLEV;
  or_hier* h = (or_hier*)calloc(1, sizeof(or_hier));
  if (!h) { *status = OR_E_NOMEM; return NULL; }
  long nnz = rp[n];
  if (csr_alloc(&h->A[0], n, nnz)) goto nomem;
  memcpy(h->A[0].rp, rp, sizeof(int) * ((size_t)n + 1));
  memcpy(h->A[0].ci, ci, sizeof(int) * (size_t)nnz);
  memcpy(h->A[0].v, v, sizeof(double) * (size_t)nnz);
  h->lu = (double*)malloc(sizeof(double) * (size_t)nnz);
  if (!h->lu) goto nomem;
  *status = or_ilu0(n, rp, ci, v, h->lu);
  if (*status) { or_free(h); return NULL; }
  if (o.ilu_k < 0) o.ilu_k = 0;
  {
    int *frp, *fci, *flev;
    double* fv;
    *status = or_iluk(n, rp, ci, v, o.ilu_k, &frp, &fci, &fv, &flev);
    if (*status) { or_free(h); return NULL; }
    h->F.n = n;
    h->F.rp = frp;
    h->F.ci = fci;
    h->F.v = fv;
    h->flev = flev;
  }
  int d = 0;
  for (;;) {
    or_csr* A = &h->A[d];
    if (A->n <= o.max_coarse || d + 1 >= o.max_levels) break;
    int* cf = (int*)malloc(sizeof(int) * (size_t)A->n);
    if (!cf) goto nomem;
    int nc = rs_split(A, o.theta, cf);
    if (nc < 0) { free(cf); goto nomem; }
    if (nc == 0 || (double)nc > 0.9 * (double)A->n) { free(cf); break; }
    h->cf[d] = cf;
    if (rs_interp(A, o.theta, cf, &h->P[d])) goto nomem;
    if (csr_transpose(&h->P[d], nc, &h->R[d])) goto nomem;
    if (galerkin(A, &h->P[d], &h->R[d], nc, &h->A[d + 1])) goto nomem;
    d++;
  }
  h->nlev = d + 1;
  h->n0 = h->A[d].n;
  h->chol = (double*)malloc(sizeof(double) * (size_t)h->n0 * (size_t)h->n0);
  if (!h->chol) goto nomem;
  *status = dense_cholesky(&h->A[d], h->chol);
  if (*status) { or_free(h); return NULL; }
  h->work = (double*)malloc(sizeof(double) * (size_t)n * 8);
  if (!h->work) goto nomem;
  h->s_scale = o.s_scale;
  h->b_scale = o.b_scale;
  *status = OR_OK;
  return h;
nomem:
  or_free(h);
  *status = OR_E_NOMEM;
  return NULL;
}

/* ------------------------------------------------------------------ */
/* Kernels of the SOLVE phase, each the plain definition. */

static void spmv(const or_csr* a, const double* x, double* y) {
  for (int i = 0; i < a->n; ++i) {
    double s = 0.0;
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) s = s + a->v[p] * x[a->ci[p]];
    y[i] = s;
  }
}

/* r = f - A u */
static void residual(const or_csr* a, const double* f, const double* u, double* r) {
  for (int i = 0; i < a->n; ++i) {
    double s = 0.0;
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) s = s + a->v[p] * u[a->ci[p]];
    r[i] = f[i] - s;
  }
}

/* y = (D+L)^{-1} f : one forward Gauss-Seidel sweep from zero */
static void forward_gs(const or_csr* a, const double* f, double* y) {
  for (int i = 0; i < a->n; ++i) {
    double s = f[i], dii = 0.0;
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
      int j = a->ci[p];
      if (j < i) s = s - a->v[p] * y[j];
      else if (j == i) dii = a->v[p];
    }
    y[i] = s / dii;
  }
}

/* y = (D+U)^{-1} f : one backward Gauss-Seidel sweep from zero; this is the
 * adjoint of forward_gs for symmetric A ((D+L)^T = D+U). */
static void backward_gs(const or_csr* a, const double* f, double* y) {
  for (int i = a->n - 1; i >= 0; --i) {
    double s = f[i], dii = 0.0;
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
      int j = a->ci[p];
      if (j > i) s = s - a->v[p] * y[j];
      else if (j == i) dii = a->v[p];
    }
    y[i] = s / dii;
  }
}

/* z = (LU)^{-1} r with the ILU(k) factors (for k = 0 on the pattern of A) */
static void ilu_apply(const or_hier* h, const double* r, double* z) {
  const or_csr* a = &h->F;
  const double* lu = h->F.v;
  int n = a->n;
  /* L y = r (unit lower) */
  for (int i = 0; i < n; ++i) {
    double s = r[i];
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p)
      if (a->ci[p] < i) s = s - lu[p] * z[a->ci[p]];
    z[i] = s;
  }
  /* U z = y */
  for (int i = n - 1; i >= 0; --i) {
    double s = z[i], uii = 0.0;
    for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
      int j = a->ci[p];
      if (j > i) s = s - lu[p] * z[j];
      else if (j == i) uii = lu[p];
    }
    z[i] = s / uii;
  }
}

/* coarsest level: e = A_0^{-1} f via the Cholesky factor */
static void coarse_solve(const or_hier* h, const double* f, double* e) {
  int n = h->n0;
  const double* g = h->chol;
  for (int i = 0; i < n; ++i) {
    double s = f[i];
    for (int k = 0; k < i; ++k) s = s - g[(long)i * n + k] * e[k];
    e[i] = s / g[(long)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = e[i];
    for (int k = i + 1; k < n; ++k) s = s - g[(long)k * n + i] * e[k];
    e[i] = s / g[(long)i * n + i];
  }
}

/* Algorithm 3.2 at depth d (paper level l = L - d) for A_l u = f with zero
 * initial guess:
 *   (1) u1 = 0 + S_l (f - A_l 0) = (D+L)^{-1} f
 *   (2a) f_{l-1} = P_{l-1}^T (f - A_l u1)
 *   (2b) coarsest: e = A_0^{-1} f_{l-1}; else e = V-cycle on level l-1 from zero
 *   (2c) u2 = u1 + P_{l-1} e
 *   (3) u3 = u2 + S_l^T (f - A_l u2), S_l^T = (D+U)^{-1}
 * A one-level hierarchy is the exact solve. */
static void vcycle(const or_hier* h, int d, const double* f, double* u) {
  if (d == h->nlev - 1) { coarse_solve(h, f, u); return; }
  const or_csr* A = &h->A[d];
  int n = A->n, nc = h->A[d + 1].n;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  double* fc = (double*)malloc(sizeof(double) * (size_t)nc);
  double* e = (double*)malloc(sizeof(double) * (size_t)nc);
  /* (1) pre-smoothing */
  forward_gs(A, f, u);
  /* (2a) restriction of the residual */
  residual(A, f, u, r);
  spmv(&h->R[d], r, fc);
  /* (2b) */
  vcycle(h, d + 1, fc, e);
  /* (2c) prolongation */
  spmv(&h->P[d], e, w);
  for (int i = 0; i < n; ++i) u[i] = u[i] + w[i];
  /* (3) post-smoothing */
  residual(A, f, u, r);
  backward_gs(A, r, w);
  for (int i = 0; i < n; ++i) u[i] = u[i] + w[i];
  free(r);
  free(w);
  free(fc);
  free(e);
}

/* The V-cycle of the AMG(ILU(0)) comparator (Section 5): as Algorithm 3.2 on the
 * finest level but with ILU(0) as the smoother, pre: u1 = (LU)^{-1} f, post:
 * u3 = u2 + (LU)^{-1} (f - A u2) (for symmetric A the ILU(0) product LU is
 * symmetric up to rounding, so the same factor serves as its own adjoint); the
 * coarser levels use the Gauss-Seidel V-cycle. A one-level hierarchy is the exact
 * solve. */
static void vcycle_ilu_top(const or_hier* h, const double* f, double* u) {
  if (h->nlev == 1) { coarse_solve(h, f, u); return; }
  const or_csr* A = &h->A[0];
  int n = A->n, nc = h->A[1].n;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  double* fc = (double*)malloc(sizeof(double) * (size_t)nc);
  double* e = (double*)malloc(sizeof(double) * (size_t)nc);
  ilu_apply(h, f, u);
  residual(A, f, u, r);
  spmv(&h->R[0], r, fc);
  vcycle(h, 1, fc, e);
  spmv(&h->P[0], e, w);
  for (int i = 0; i < n; ++i) u[i] = u[i] + w[i];
  residual(A, f, u, r);
  ilu_apply(h, r, w);
  for (int i = 0; i < n; ++i) u[i] = u[i] + w[i];
  free(r);
  free(w);
  free(fc);
  free(e);
}

typedef void (*op_fn)(const or_hier* h, const double* r, double* z);

static void op_vcycle(const or_hier* h, const double* r, double* z) { vcycle(h, 0, r, z); }
static void op_ilu(const or_hier* h, const double* r, double* z) { ilu_apply(h, r, z); }
static void op_fgs(const or_hier* h, const double* r, double* z) { forward_gs(&h->A[0], r, z); }
static void op_bgs(const or_hier* h, const double* r, double* z) { backward_gs(&h->A[0], r, z); }

/* Algorithm 2.1 from u^{k,0} = 0:
 *   (1) u1 = 0 + S f
 *   (2) u2 = u1 + B (f - A u1)
 *   (3) u3 = u2 + S^T (f - A u2) */
static void combined(const or_hier* h, op_fn S, op_fn B, op_fn ST, const double* f, double* u) {
  const or_csr* A = &h->A[0];
  int n = A->n;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  S(h, f, u);
  if (h->s_scale != 1.0) for (int i = 0; i < n; ++i) u[i] = h->s_scale * u[i];
  residual(A, f, u, r);
  B(h, r, w);
  if (h->b_scale != 1.0) for (int i = 0; i < n; ++i) w[i] = h->b_scale * w[i];
  for (int i = 0; i < n; ++i) u[i] = u[i] + w[i];
  residual(A, f, u, r);
  ST(h, r, w);
  if (h->s_scale != 1.0) for (int i = 0; i < n; ++i) w[i] = h->s_scale * w[i];
  for (int i = 0; i < n; ++i) u[i] = u[i] + w[i];
  free(r);
  free(w);
}

/* S~ f for S = V-cycle: (I - S~A) = (I - S^T A)(I - S A), i.e. two cycles:
 * u1 = S f, u2 = u1 + S^T (f - A u1); S^T = S because the cycle is symmetric. */
static void sym_smoother(const or_hier* h, const double* f, double* u) {
  const or_csr* A = &h->A[0];
  int n = A->n;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  vcycle(h, 0, f, u);
  residual(A, f, u, r);
  vcycle(h, 0, r, w);
  for (int i = 0; i < n; ++i) u[i] = u[i] + w[i];
  free(r);
  free(w);
}

/* AMG(ILU(0)) with two cycles: z = V'(f), z = z + V'(f - A z), V' = vcycle_ilu_top */
static void amg_ilu(const or_hier* h, const double* f, double* u) {
  const or_csr* A = &h->A[0];
  int n = A->n;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  vcycle_ilu_top(h, f, u);
  residual(A, f, u, r);
  vcycle_ilu_top(h, r, w);
  for (int i = 0; i < n; ++i) u[i] = u[i] + w[i];
  free(r);
  free(w);
}

/* B-bar of the remark after Theorem 2.1, I - B-bar A = (I - BA)(I - S~A)(I - BA),
 * applied to f from a zero start: the error propagators act right to left, so
 *   u1 = B f,  u2 = u1 + S~ (f - A u1),  u3 = u2 + B (f - A u2),
 * with B = b_scale * ILU(0) and S~ the two-cycle AMG(GS) operator. */
static void bbar(const or_hier* h, const double* f, double* u) {
  const or_csr* A = &h->A[0];
  int n = A->n;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  ilu_apply(h, f, u);
  for (int i = 0; i < n; ++i) u[i] = h->b_scale * u[i];
  residual(A, f, u, r);
  sym_smoother(h, r, w);
  for (int i = 0; i < n; ++i) u[i] = u[i] + w[i];
  residual(A, f, u, r);
  ilu_apply(h, r, w);
  for (int i = 0; i < n; ++i) u[i] = u[i] + h->b_scale * w[i];
  free(r);
  free(w);
}

int or_apply(const or_hier* h, int which, const double* r, double* z) {
  int n = h->A[0].n;
  switch (which) {
    case OR_PREC_COMBINED: combined(h, op_vcycle, op_ilu, op_vcycle, r, z); return OR_OK;
    case OR_PREC_AMG: sym_smoother(h, r, z); return OR_OK;
    case OR_PREC_ILU: ilu_apply(h, r, z); return OR_OK;
    case OR_PREC_ADDITIVE: {
      double* w = (double*)malloc(sizeof(double) * (size_t)n);
      sym_smoother(h, r, z);
      ilu_apply(h, r, w);
      for (int i = 0; i < n; ++i) z[i] = z[i] + h->b_scale * w[i];
      free(w);
      return OR_OK;
    }
    case OR_PREC_NONE: memcpy(z, r, sizeof(double) * (size_t)n); return OR_OK;
    case OR_OP_VCYCLE: vcycle(h, 0, r, z); return OR_OK;
    case OR_OP_FGS: forward_gs(&h->A[0], r, z); return OR_OK;
    case OR_OP_BGS: backward_gs(&h->A[0], r, z); return OR_OK;
    case OR_OP_COMBINED_GS: combined(h, op_fgs, op_ilu, op_bgs, r, z); return OR_OK;
    case OR_OP_COMBINED_SWAP: combined(h, op_ilu, op_vcycle, op_ilu, r, z); return OR_OK;
    case OR_PREC_AMG_ILU: amg_ilu(h, r, z); return OR_OK;
    case OR_PREC_BBAR: bbar(h, r, z); return OR_OK;
    default: return OR_E_ARG;
  }
}

static double dot(int n, const double* x, const double* y) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s = s + x[i] * y[i];
  return s;
}

/* Preconditioned conjugate gradients for A x = b with preconditioner `which`.
 * x holds the initial guess when use_x0 != 0, else starts from 0.
 * Stops when ||r_k||_2 / ||b||_2 <= tol on the recursively updated residual
 * (checked before the first iteration too) or after maxit iterations.
 * hist[k] = ||r_k|| / ||b|| for k = 0..iters (caller array of maxit+1, or NULL).
 * true_relres = ||b - A x|| / ||b|| at exit. b = 0 gives x = 0, iters = 0. */
int or_pcg(const or_hier* h, int which, const double* b, double* x, int use_x0, double tol, int maxit,
           int* iters, double* hist, double* true_relres) {
  const or_csr* A = &h->A[0];
  int n = A->n;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* z = (double*)malloc(sizeof(double) * (size_t)n);
  double* p = (double*)malloc(sizeof(double) * (size_t)n);
  double* q = (double*)malloc(sizeof(double) * (size_t)n);
  int status = OR_OK;
  *iters = 0;
  double bnorm = sqrt(dot(n, b, b));
  if (bnorm == 0.0) {
    for (int i = 0; i < n; ++i) x[i] = 0.0;
    if (hist) hist[0] = 0.0;
    *true_relres = 0.0;
    goto done;
  }
  if (use_x0) residual(A, b, x, r);
  else {
    for (int i = 0; i < n; ++i) x[i] = 0.0;
    memcpy(r, b, sizeof(double) * (size_t)n);
  }
  double rel = sqrt(dot(n, r, r)) / bnorm;
  if (hist) hist[0] = rel;
  if (rel <= tol) goto finish;
  or_apply(h, which, r, z);
  memcpy(p, z, sizeof(double) * (size_t)n);
  double rz = dot(n, r, z);
  if (!(rz > 0.0)) { status = OR_E_BREAKDOWN; goto finish; }
  int k;
  for (k = 1; k <= maxit; ++k) {
    spmv(A, p, q);
    double pq = dot(n, p, q);
    if (!(pq > 0.0)) { status = OR_E_BREAKDOWN; *iters = k - 1; goto finish; }
    double alpha = rz / pq;
    for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
    for (int i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
    rel = sqrt(dot(n, r, r)) / bnorm;
    if (hist) hist[k] = rel;
    *iters = k;
    if (!isfinite(rel)) { status = OR_E_BREAKDOWN; goto finish; }
    if (rel <= tol) goto finish;
    if (k == maxit) break;
    or_apply(h, which, r, z);
    double rz_new = dot(n, r, z);
    if (!(rz_new > 0.0)) { status = OR_E_BREAKDOWN; goto finish; }
    double beta = rz_new / rz;
    rz = rz_new;
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  status = OR_E_MAXIT;
finish:
  residual(A, b, x, r);
  *true_relres = sqrt(dot(n, r, r)) / bnorm;
done:
  free(r);
  free(z);
  free(p);
  free(q);
  return status;
}

/* ------------------------------------------------------------------ */
/* accessors for the Python wrapper (depth d = 0 is the finest level) */
int or_nlev(const or_hier* h) { return h->nlev; }
int or_level_n(const or_hier* h, int d) { return h->A[d].n; }
long or_level_nnz(const or_hier* h, int d) { return h->A[d].rp[h->A[d].n]; }
long or_p_nnz(const or_hier* h, int d) { return (d < h->nlev - 1) ? h->P[d].rp[h->P[d].n] : 0; }
void or_get_level(const or_hier* h, int d, int* rp, int* ci, double* v) {
  const or_csr* a = &h->A[d];
  memcpy(rp, a->rp, sizeof(int) * ((size_t)a->n + 1));
  memcpy(ci, a->ci, sizeof(int) * (size_t)a->rp[a->n]);
  memcpy(v, a->v, sizeof(double) * (size_t)a->rp[a->n]);
}
void or_get_p(const or_hier* h, int d, int* rp, int* ci, double* v) {
  const or_csr* a = &h->P[d];
  memcpy(rp, a->rp, sizeof(int) * ((size_t)a->n + 1));
  memcpy(ci, a->ci, sizeof(int) * (size_t)a->rp[a->n]);
  memcpy(v, a->v, sizeof(double) * (size_t)a->rp[a->n]);
}
void or_get_cf(const or_hier* h, int d, int* cf) { memcpy(cf, h->cf[d], sizeof(int) * (size_t)h->A[d].n); }
void or_get_ilu(const or_hier* h, double* lu) { memcpy(lu, h->lu, sizeof(double) * (size_t)h->A[0].rp[h->A[0].n]); }
long or_ilu_nnz(const or_hier* h) { return h->F.rp[h->F.n]; }
void or_get_ilu_factor(const or_hier* h, int* rp, int* ci, double* v, int* lev) {
  long nnz = h->F.rp[h->F.n];
  memcpy(rp, h->F.rp, sizeof(int) * ((size_t)h->F.n + 1));
  memcpy(ci, h->F.ci, sizeof(int) * (size_t)nnz);
  memcpy(v, h->F.v, sizeof(double) * (size_t)nnz);
  memcpy(lev, h->flev, sizeof(int) * (size_t)nnz);
}
void or_get_chol(const or_hier* h, double* g) { memcpy(g, h->chol, sizeof(double) * (size_t)h->n0 * (size_t)h->n0); }

/* standalone pieces for pins */
int or_rs_split(int n, const int* rp, const int* ci, const double* v, double theta, int* cf) {
  or_csr a = {n, (int*)rp, (int*)ci, (double*)v};
  return rs_split(&a, theta, cf);
}
