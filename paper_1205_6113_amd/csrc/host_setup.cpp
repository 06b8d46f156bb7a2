// Host-side SETUP: validation, ILU(0), classical coarsening/interpolation,
// sweep schedules, exact coarsest solve. Compiled without FMA contraction so
// that every product and sum is rounded on its own (the coarsening decisions
// compare values against thresholds, so the arithmetic order is fixed and
// documented at each function).
#include "host_setup.hpp"

#include <algorithm>
#include <tuple>
#include <thread>
#include <atomic>
#include <queue>
#include <map>
#include <functional>
#include <cmath>
#include <cstring>
#include <limits>

#include "../../include/cpc.h"

namespace cpc {

int validate_csr(int n, const int32_t* rp, const int32_t* ci, const double* v, bool check_symmetry,
                 std::string* msg) {
  auto fail = [&](int code, const std::string& m) {
    if (msg) *msg = m;
    return code;
  };
  if (n <= 0) return fail(CPC_E_ARG, "n must be positive");
  if (!rp || !ci || !v) return fail(CPC_E_ARG, "null CSR array");
  if (rp[0] != 0) return fail(CPC_E_ARG, "row_ptr[0] must be 0");
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return fail(CPC_E_ARG, "row_ptr not monotone at row " + std::to_string(i));
    bool diag = false;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      if (j < 0 || j >= n) return fail(CPC_E_ARG, "column out of range in row " + std::to_string(i));
      if (p > rp[i] && j <= ci[p - 1]) return fail(CPC_E_ARG, "columns not sorted/unique in row " + std::to_string(i));
      if (!std::isfinite(v[p])) return fail(CPC_E_ARG, "non-finite value in row " + std::to_string(i));
      if (j == i) {
        diag = true;
        if (!(v[p] > 0.0)) return fail(CPC_E_NOT_SPD, "non-positive diagonal at row " + std::to_string(i));
      }
    }
    if (!diag) return fail(CPC_E_ARG, "missing diagonal in row " + std::to_string(i));
  }
  if (check_symmetry) {
    for (int i = 0; i < n; ++i)
      for (int p = rp[i]; p < rp[i + 1]; ++p) {
        int j = ci[p];
        const int32_t* b = ci + rp[j];
        const int32_t* e = ci + rp[j + 1];
        const int32_t* it = std::lower_bound(b, e, i);
        if (it == e || *it != i) return fail(CPC_E_ARG, "pattern not symmetric at (" + std::to_string(i) + "," + std::to_string(j) + ")");
        double x = v[p], y = v[rp[j] + (it - b)];
        if (std::fabs(x - y) > 1e-12 * std::max(std::fabs(x), std::fabs(y)))
          return fail(CPC_E_ARG, "values not symmetric at (" + std::to_string(i) + "," + std::to_string(j) + ")");
      }
  }
  return CPC_OK;
}

// ILU(0): row i is reduced by every earlier row m it couples to, in increasing m;
// the multiplier l_im = a_im / u_mm overwrites a_im and a_ij -= l_im * u_mj for the
// j > m of row m that are in the pattern of row i (all other fill is dropped).
int ilu0_factor(const HostCsr& a, std::vector<double>& lu, std::string* msg) {
  const int n = a.n;
  lu = a.v;
  std::vector<int> where(n, -1), dpos(n, -1);
  for (int i = 0; i < n; ++i) {
    const int b = a.rp[i], e = a.rp[i + 1];
    for (int p = b; p < e; ++p) {
      where[a.ci[p]] = p;
      if (a.ci[p] == i) dpos[i] = p;
    }
    for (int p = b; p < e; ++p) {
      const int m = a.ci[p];
      if (m >= i) break;
      const double l = lu[p] / lu[dpos[m]];
      lu[p] = l;
      for (int q = dpos[m] + 1; q < a.rp[m + 1]; ++q) {
        const int t = where[a.ci[q]];
        if (t >= 0) lu[t] = lu[t] - l * lu[q];
      }
    }
    for (int p = b; p < e; ++p) where[a.ci[p]] = -1;
    if (!(lu[dpos[i]] > 0.0)) {
      if (msg) *msg = "ILU(0) pivot not positive at row " + std::to_string(i);
      return CPC_E_NOT_SPD;
    }
  }
  return CPC_OK;
}

int iluk_factor(const HostCsr& a, int k, HostCsr& f, std::vector<int>& lev, std::string* msg) {
  // Row i: values and levels in dense arrays over the columns touched so far; the
  // pivots still to visit (columns below i) in a min-heap, so that they are taken in
  // increasing order even as eliminations add new ones. A pivot m whose level exceeds
  // k is passed over; entry (i, j) of row m of the factor updates (i, j) as
  // w_j - w_m u_mj (a new entry enters as 0), with level min(lev_j, lev_m + lev_mj + 1).
  // Entries above level k are dropped when the row is done.
  constexpr int kInf = 1 << 28;
  const int n = a.n;
  f = HostCsr{};
  f.n = n;
  f.ncols = n;
  f.rp.assign(n + 1, 0);
  f.ci.reserve(a.ci.size() + n);
  f.v.reserve(a.ci.size() + n);
  lev.clear();
  lev.reserve(a.ci.size() + n);
  std::vector<double> w(n, 0.0);
  std::vector<int> lv(n, -1), dpos(n, -1), touched;
  std::vector<int> heap;
  auto later = std::greater<int>();
  for (int i = 0; i < n; ++i) {
    touched.clear();
    heap.clear();
    for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) {
      const int j = a.ci[p];
      w[j] = a.v[p];
      lv[j] = 0;
      touched.push_back(j);
      if (j < i) heap.push_back(j);
    }
    std::make_heap(heap.begin(), heap.end(), later);
    while (!heap.empty()) {
      std::pop_heap(heap.begin(), heap.end(), later);
      const int m = heap.back();
      heap.pop_back();
      if (lv[m] > k) continue;
      w[m] = w[m] / f.v[dpos[m]];
      for (int q = dpos[m] + 1; q < f.rp[m + 1]; ++q) {
        const int j = f.ci[q];
        if (lv[j] < 0) {
          w[j] = 0.0;
          lv[j] = kInf;
          touched.push_back(j);
          if (j < i) {
            heap.push_back(j);
            std::push_heap(heap.begin(), heap.end(), later);
          }
        }
        w[j] = w[j] - w[m] * f.v[q];
        const int l = lv[m] + lev[q] + 1;
        if (l < lv[j]) lv[j] = l;
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int j : touched) {
      if (lv[j] <= k) {
        if (j == i) dpos[i] = (int)f.ci.size();
        f.ci.push_back(j);
        f.v.push_back(w[j]);
        lev.push_back(lv[j]);
      }
      lv[j] = -1;
    }
    f.rp[i + 1] = (int)f.ci.size();
    if (dpos[i] < 0 || !(f.v[dpos[i]] > 0.0)) {
      if (msg) *msg = "ILU(" + std::to_string(k) + ") pivot not positive at row " + std::to_string(i);
      return CPC_E_NOT_SPD;
    }
  }
  return CPC_OK;
}

namespace {

// strong couplings of each row (CSR of column indices) and their transpose
struct Graph {
  std::vector<int> rp, ci;
};

void strength(const HostCsr& a, double theta, Graph& S, Graph& ST) {
  const int n = a.n;
  S.rp.assign(n + 1, 0);
  S.ci.clear();
  S.ci.reserve(a.nnz());
  for (int i = 0; i < n; ++i) {
    bool have = false;
    double mx = 0.0;
    for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) {
      if (a.ci[p] == i) continue;
      const double t = -a.v[p];
      if (!have || t > mx) mx = t;
      have = true;
    }
    const double thr = theta * mx;
    for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) {
      const int j = a.ci[p];
      if (j != i && a.v[p] < 0.0 && -a.v[p] >= thr) S.ci.push_back(j);
    }
    S.rp[i + 1] = (int)S.ci.size();
  }
  ST.rp.assign(n + 1, 0);
  ST.ci.assign(S.ci.size(), 0);
  for (int j : S.ci) ST.rp[j + 1]++;
  for (int i = 0; i < n; ++i) ST.rp[i + 1] += ST.rp[i];
  std::vector<int> next(ST.rp.begin(), ST.rp.end() - 1);
  for (int i = 0; i < n; ++i)
    for (int p = S.rp[i]; p < S.rp[i + 1]; ++p) ST.ci[next[S.ci[p]]++] = i;
}

// max-tree over points: key = lambda for undecided points, -1 otherwise;
// the root holds the largest key and, among equal keys, the smallest index.
class MaxTree {
 public:
  explicit MaxTree(int n) : n_(n) {
    size_ = 1;
    while (size_ < n) size_ <<= 1;
    key_.assign(2 * size_, -1);
    idx_.assign(2 * size_, std::numeric_limits<int>::max());
    for (int i = 0; i < n; ++i) idx_[size_ + i] = i;
  }
  void set(int i, int key) {
    int t = size_ + i;
    key_[t] = key;
    for (t >>= 1; t >= 1; t >>= 1) pull(t);
  }
  void build() {
    for (int t = size_ - 1; t >= 1; --t) pull(t);
  }
  void set_leaf(int i, int key) { key_[size_ + i] = key; }
  int top_key() const { return key_[1]; }
  int top_idx() const { return idx_[1]; }

 private:
  void pull(int t) {
    const int l = 2 * t, r = l + 1;
    if (key_[l] >= key_[r]) {
      key_[t] = key_[l];
      idx_[t] = idx_[l];
    } else {
      key_[t] = key_[r];
      idx_[t] = idx_[r];
    }
  }
  int n_, size_;
  std::vector<int> key_, idx_;
};

}  // namespace

// Classical coarsening. Strength: j in S_i iff a_ij < 0 and -a_ij >= theta * max_k(-a_ik).
// First pass: points with no strong couplings are F; the undecided point with the
// largest lambda_i = |S_i^T among undecided| (smallest index on ties) becomes C, the
// undecided points of S_i^T become F (each raising lambda of the undecided points of
// its own S_j), then the undecided points of S_i lose one from lambda.
// Second pass over F points in increasing index: a strong F neighbour j with no strong
// coupling into C_i becomes the tentative C point; a second such j turns i itself into
// C (the tentative point is dropped); a surviving tentative point becomes C.
int rs_coarsen(const HostCsr& a, double theta, std::vector<int>& cf) {
  const int n = a.n;
  Graph S, ST;
  strength(a, theta, S, ST);
  constexpr int UNDECIDED = -1, F = 0, C = 1;
  cf.assign(n, UNDECIDED);
  for (int i = 0; i < n; ++i)
    if (S.rp[i] == S.rp[i + 1]) cf[i] = F;
  std::vector<int> lambda(n, 0);
  MaxTree tree(n);
  for (int i = 0; i < n; ++i) {
    if (cf[i] != UNDECIDED) continue;
    int c = 0;
    for (int p = ST.rp[i]; p < ST.rp[i + 1]; ++p) c += (cf[ST.ci[p]] == UNDECIDED);
    lambda[i] = c;
    tree.set_leaf(i, c);
  }
  tree.build();
  while (tree.top_key() >= 0) {
    const int i = tree.top_idx();
    cf[i] = C;
    tree.set(i, -1);
    for (int p = ST.rp[i]; p < ST.rp[i + 1]; ++p) {
      const int j = ST.ci[p];
      if (cf[j] != UNDECIDED) continue;
      cf[j] = F;
      tree.set(j, -1);
      for (int q = S.rp[j]; q < S.rp[j + 1]; ++q) {
        const int k = S.ci[q];
        if (cf[k] == UNDECIDED) tree.set(k, ++lambda[k]);
      }
    }
    for (int p = S.rp[i]; p < S.rp[i + 1]; ++p) {
      const int j = S.ci[p];
      if (cf[j] == UNDECIDED) tree.set(j, --lambda[j]);
    }
  }
  // second pass
  std::vector<int> owner(n, -1);  // owner[k] == i : k belongs to C_i of the F point i
  for (int i = 0; i < n; ++i) {
    if (cf[i] != F) continue;
    for (int p = S.rp[i]; p < S.rp[i + 1]; ++p)
      if (cf[S.ci[p]] == C) owner[S.ci[p]] = i;
    int tentative = -1;
    bool promoted = false;
    for (int p = S.rp[i]; p < S.rp[i + 1] && !promoted; ++p) {
      const int j = S.ci[p];
      if (cf[j] != F) continue;
      bool covered = false;
      for (int q = S.rp[j]; q < S.rp[j + 1]; ++q)
        if (owner[S.ci[q]] == i) {
          covered = true;
          break;
        }
      if (covered) continue;
      if (tentative < 0) {
        tentative = j;
        owner[j] = i;
      } else {
        cf[i] = C;
        promoted = true;
      }
    }
    if (!promoted && tentative >= 0) cf[tentative] = C;
  }
  int nc = 0;
  for (int i = 0; i < n; ++i) nc += (cf[i] == C);
  return nc;
}

// Classical interpolation. For an F point i, C_i = strong C neighbours, D^s_i =
// strong F neighbours, D^w_i = all other off-diagonals (weak, or a strong F neighbour
// m whose sum over C_i of abar_mk is zero; abar_mk = a_mk when its sign is opposite
// to a_mm, else 0):
//   w_ij = -(a_ij + sum_{m in D^s_i} (a_im * abar_mj) / d_m) / (a_ii + sum_{n in D^w_i} a_in),
//   d_m = sum_{k in C_i} abar_mk.
// Sums run in increasing column order; each numerator starts from a_ij and adds the
// m terms in increasing m; d_m starts from 0. C points get a unit row; points with
// no strong couplings get an empty row.
bool rs_interpolation(const HostCsr& a, double theta, const std::vector<int>& cf, int nc, HostCsr& P) {
  const int n = a.n;
  Graph S, ST;
  strength(a, theta, S, ST);
  std::vector<int> coarse(n, -1);
  {
    int c = 0;
    for (int i = 0; i < n; ++i)
      if (cf[i] == 1) coarse[i] = c++;
  }
  std::vector<double> diag(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int p = a.rp[i]; p < a.rp[i + 1]; ++p)
      if (a.ci[p] == i) diag[i] = a.v[p];
  P.n = n;
  P.ncols = nc;
  P.rp.assign(n + 1, 0);
  P.ci.clear();
  P.v.clear();
  // role[k] for the F point being processed: 1 = C_i, 2 = D^s_i (kept), 3 = D^s_i moved to D^w
  std::vector<uint8_t> role(n, 0);
  std::vector<double> num(n, 0.0);
  std::vector<double> dm;  // d_m per strong F neighbour, in S_i order
  for (int i = 0; i < n; ++i) {
    if (cf[i] == 1) {
      P.ci.push_back(coarse[i]);
      P.v.push_back(1.0);
      P.rp[i + 1] = (int)P.ci.size();
      continue;
    }
    const int sb = S.rp[i], se = S.rp[i + 1];
    for (int p = sb; p < se; ++p) role[S.ci[p]] = (cf[S.ci[p]] == 1) ? 1 : 2;
    auto dsum_of = [&](int m) {
      const bool neg_diag = diag[m] < 0.0;
      double d = 0.0;
      for (int q = a.rp[m]; q < a.rp[m + 1]; ++q) {
        const int k = a.ci[q];
        if (k != m && role[k] == 1 && ((a.v[q] < 0.0) != neg_diag)) d = d + a.v[q];
      }
      return d;
    };
    for (int p = sb; p < se; ++p) {
      const int m = S.ci[p];
      if (role[m] == 2 && dsum_of(m) == 0.0) role[m] = 3;
    }
    double denom = diag[i];
    for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) {
      const int k = a.ci[p];
      if (k == i || role[k] == 1 || role[k] == 2) continue;
      denom = denom + a.v[p];
    }
    for (int p = a.rp[i]; p < a.rp[i + 1]; ++p)
      if (role[a.ci[p]] == 1) num[a.ci[p]] = a.v[p];
    for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) {
      const int m = a.ci[p];
      if (role[m] != 2) continue;
      const double aim = a.v[p];
      const double d = dsum_of(m);
      const bool neg_diag = diag[m] < 0.0;
      for (int q = a.rp[m]; q < a.rp[m + 1]; ++q) {
        const int j = a.ci[q];
        if (j == m || role[j] != 1 || ((a.v[q] < 0.0) == neg_diag)) continue;
        double t = aim * a.v[q];
        t = t / d;
        num[j] = num[j] + t;
      }
    }
    for (int p = sb; p < se; ++p) {
      const int j = S.ci[p];
      if (role[j] == 1) {
        P.ci.push_back(coarse[j]);
        P.v.push_back(-(num[j] / denom));
      }
    }
    P.rp[i + 1] = (int)P.ci.size();
    for (int p = sb; p < se; ++p) role[S.ci[p]] = 0;
  }
  return true;
}

HostCsr transpose(const HostCsr& a) {
  HostCsr t;
  t.n = a.ncols;
  t.ncols = a.n;
  t.rp.assign(t.n + 1, 0);
  const int64_t nnz = a.nnz();
  t.ci.resize(nnz);
  t.v.resize(nnz);
  for (int64_t p = 0; p < nnz; ++p) t.rp[a.ci[p] + 1]++;
  for (int j = 0; j < t.n; ++j) t.rp[j + 1] += t.rp[j];
  std::vector<int> next(t.rp.begin(), t.rp.end() - 1);
  for (int i = 0; i < a.n; ++i)
    for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) {
      const int q = next[a.ci[p]]++;
      t.ci[q] = i;
      t.v[q] = a.v[p];
    }
  return t;
}

int lower_depth(const HostCsr& a) {
  std::vector<int> lev(a.n, 0);
  int depth = 0;
  for (int i = 0; i < a.n; ++i) {
    int l = 0;
    for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) {
      const int j = a.ci[p];
      if (j >= i) break;
      l = std::max(l, lev[j] + 1);
    }
    lev[i] = l;
    depth = std::max(depth, l + 1);
  }
  return depth;
}

std::vector<int> sweep_block_starts(const HostCsr& a, int R, const std::vector<int>* parts) {
  const int n = a.n;
  if (n <= 0) return {0, 0};
  R = std::max(1, std::min(R, n));
  const bool use_parts = parts && parts->size() >= 2 && parts->front() == 0 && parts->back() == n;
  const std::vector<int> pr = use_parts ? *parts : std::vector<int>{0, n};
  std::vector<int> starts{0};
  for (size_t q = 0; q + 1 < pr.size(); ++q) {
    const int end = pr[q + 1];
    if (end <= starts.back()) continue;
    while (starts.back() + R < end) {
      const int s0 = starts.back();
      int cut = s0 + R;
      // prefer a row with no coupling to its predecessor
      for (int i = s0 + R; i > s0 + R / 2; --i) {
        bool coupled = false;
        for (int p = a.rp[i]; p < a.rp[i + 1] && a.ci[p] < i; ++p) coupled |= (a.ci[p] == i - 1);
        if (!coupled) {
          cut = i;
          break;
        }
      }
      starts.push_back(cut);
    }
    starts.push_back(end);
  }
  if (starts.back() != n) starts.push_back(n);
  return starts;
}

SweepSchedule build_sweep(const HostCsr& a, bool forward, int R, int64_t max_entries,
                          const std::vector<int>* parts) {
  SweepSchedule s;
  const int n = a.n;
  s.n = n;
  s.forward = forward;
  s.blk_row = sweep_block_starts(a, R, parts);
  s.nblk = (int)s.blk_row.size() - 1;
  s.R = 0;
  for (int b = 0; b < s.nblk; ++b) s.R = std::max(s.R, s.blk_row[b + 1] - s.blk_row[b]);
  std::vector<int> blk_of(n);
  for (int b = 0; b < s.nblk; ++b)
    for (int i = s.blk_row[b]; i < s.blk_row[b + 1]; ++i) blk_of[i] = b;
  std::vector<int> lev(n, 0), glev(n, 0), ndep(n, 0);
  for (int i = 0; i < n; ++i)
    for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) ndep[i] += forward ? (a.ci[p] < i) : (a.ci[p] > i);
  // global depth of every row in the sweep's own direction
  if (forward) {
    for (int i = 0; i < n; ++i) {
      int g = 0;
      for (int p = a.rp[i]; p < a.rp[i + 1] && a.ci[p] < i; ++p) g = std::max(g, glev[a.ci[p]] + 1);
      glev[i] = g;
      s.global_depth = std::max(s.global_depth, g + 1);
    }
  } else {
    for (int i = n - 1; i >= 0; --i) {
      int g = 0;
      for (int p = a.rp[i + 1] - 1; p >= a.rp[i] && a.ci[p] > i; --p) g = std::max(g, glev[a.ci[p]] + 1);
      glev[i] = g;
      s.global_depth = std::max(s.global_depth, g + 1);
    }
  }
  s.blk_beg.assign(s.nblk, 0);
  s.blk_end.assign(s.nblk, 0);
  s.perm.reserve(n);
  s.lvl_ptr.push_back(0);
  s.wait_ptr.push_back(0);
  std::vector<int> last_need(s.nblk, 0);  // running maximum of waits of the current block
  std::vector<int> touched, uniq;
  std::vector<std::vector<int>> rows_at;
  // per-level: list of (block, need) candidates
  std::vector<std::vector<std::pair<int, int>>> waits_at;
  std::vector<std::vector<int>> needs_of_block(s.nblk);  // needs placed on each block
  for (int t = 0; t < s.nblk; ++t) {
    // blocks in processing order: increasing rows forward, decreasing backward
    const int b = forward ? t : s.nblk - 1 - t;
    const int r0 = s.blk_row[b], r1 = s.blk_row[b + 1];
    // Local levels: the distinct global depths of the block's rows, in increasing
    // order. A row then waits for nothing that the global level schedule would not
    // also wait for, so blocks that run side by side advance in step; levels built
    // from the block's own rows alone let an early local level stall on a deep
    // external row and serialise the blocks behind it.
    uniq.assign(glev.begin() + r0, glev.begin() + r1);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    const int nu = (int)uniq.size();
    for (int i = r0; i < r1; ++i) lev[i] = (int)(std::lower_bound(uniq.begin(), uniq.end(), glev[i]) - uniq.begin());
    rows_at.assign(nu, {});
    for (int i = r0; i < r1; ++i) rows_at[lev[i]].push_back(i);
    // cut levels with too many dependency entries (rows of one level are independent)
    {
      std::vector<std::vector<int>> cut;
      for (auto& rows : rows_at) {
        cut.emplace_back();
        int64_t ent = 0;
        for (int i : rows) {
          const int64_t e = ndep[i];
          if (max_entries > 0 && !cut.back().empty() && ent + e > max_entries) {
            cut.emplace_back();
            ent = 0;
          }
          cut.back().push_back(i);
          ent += e;
        }
      }
      rows_at.swap(cut);
      for (auto& rows : rows_at) {
        if (rows.size() < 2) continue;
        int64_t ent = 0;
        for (int i : rows) ent += ndep[i];
        s.max_level_entries = std::max(s.max_level_entries, ent);
      }
    }
    const int nl = (int)rows_at.size();
    for (int m = 0; m < nl; ++m)
      for (int i : rows_at[m]) lev[i] = m;
    waits_at.assign(nl, {});
    for (int i = r0; i < r1; ++i) {
      if (forward) {
        for (int p = a.rp[i]; p < a.rp[i + 1] && a.ci[p] < r0; ++p) {
          const int j = a.ci[p];
          waits_at[lev[i]].push_back({blk_of[j], lev[j] + 1});
        }
      } else {
        for (int p = a.rp[i + 1] - 1; p >= a.rp[i] && a.ci[p] >= r1; --p) {
          const int j = a.ci[p];
          waits_at[lev[i]].push_back({blk_of[j], lev[j] + 1});
        }
      }
    }
    s.blk_beg[b] = (int)s.lvl_ptr.size() - 1;
    touched.clear();
    for (int m = 0; m < nl; ++m) {
      for (int i : rows_at[m]) s.perm.push_back(i);
      s.lvl_ptr.push_back((int)s.perm.size());
      auto& w = waits_at[m];
      std::sort(w.begin(), w.end());
      for (size_t t = 0; t < w.size(); ++t) {
        if (t + 1 < w.size() && w[t + 1].first == w[t].first) continue;  // keep the largest need per block
        const int ob = w[t].first, need = w[t].second;
        if (need > last_need[ob]) {
          if (last_need[ob] == 0) touched.push_back(ob);
          last_need[ob] = need;
          s.wait_blk.push_back(ob);
          s.wait_need.push_back(need);
          needs_of_block[ob].push_back(need);
        }
      }
      s.wait_ptr.push_back((int)s.wait_blk.size());
    }
    for (int ob : touched) last_need[ob] = 0;
    s.blk_end[b] = (int)s.lvl_ptr.size() - 1;
    s.max_local_levels = std::max(s.max_local_levels, nl);
  }
  const int total = (int)s.lvl_ptr.size() - 1;
  s.publish.assign(total, 0);
  for (int b = 0; b < s.nblk; ++b)
    for (int need : needs_of_block[b]) s.publish[s.blk_beg[b] + need - 1] = 1;
  return s;
}

int dominant_stride(const HostCsr& a) {
  std::map<int, int> count;
  for (int i = 0; i < a.n; ++i)
    if (a.rp[i] < a.rp[i + 1] && a.ci[a.rp[i]] < i) ++count[i - a.ci[a.rp[i]]];
  int best = 0, bc = 0;
  for (const auto& kv : count)
    if (kv.second > bc) {
      best = kv.first;
      bc = kv.second;
    }
  return best;
}

bool build_wave_schedule(const HostCsr& a, bool forward, int W, int M, int stride, WaveSchedule& s) {
  const int n = a.n;
  if (W < 1 || M < 1) return false;
  if (M > 1 && stride < W) M = 1;  // segments would overlap: contiguous blocks
  s = WaveSchedule{};
  s.forward = forward;
  s.n = n;
  s.W = W;
  s.M = M;
  s.stride = M > 1 ? stride : 0;
  // global depth of every row in the solve's direction
  std::vector<int> depth(n, 0);
  if (forward) {
    for (int i = 0; i < n; ++i) {
      int g = 0;
      for (int q = a.rp[i]; q < a.rp[i + 1] && a.ci[q] < i; ++q) g = std::max(g, depth[a.ci[q]] + 1);
      depth[i] = g;
      s.global_depth = std::max(s.global_depth, g + 1);
    }
  } else {
    for (int i = n - 1; i >= 0; --i) {
      int g = 0;
      for (int q = a.rp[i + 1] - 1; q >= a.rp[i] && a.ci[q] > i; --q) g = std::max(g, depth[a.ci[q]] + 1);
      depth[i] = g;
      s.global_depth = std::max(s.global_depth, g + 1);
    }
  }
  // block of each row (keys in increasing order of their first row)
  const int64_t nr = M > 1 ? (stride + W - 1) / W : 0;
  auto key = [&](int i) -> int64_t {
    if (M == 1) return i / W;
    return ((int64_t)i / ((int64_t)stride * M)) * nr + (i % stride) / W;
  };
  std::map<int64_t, int> ids;
  std::vector<int> blk(n), first;
  for (int i = 0; i < n; ++i) {
    auto it = ids.find(key(i));
    if (it == ids.end()) {
      it = ids.emplace(key(i), (int)first.size()).first;
      first.push_back(i);
    }
    blk[i] = it->second;
  }
  const int nb = (int)first.size();
  std::vector<int> last(nb, 0), cnt(nb, 0);
  for (int i = 0; i < n; ++i) {
    last[blk[i]] = i;
    ++cnt[blk[i]];
  }
  // dependency graph between blocks and a topological order of it (forward: earliest
  // first row first; backward: latest last row first)
  std::vector<std::vector<int>> succ(nb);
  std::vector<int> indeg(nb, 0);
  {
    for (int i = 0; i < n; ++i) {
      const int bi = blk[i];
      for (int q = a.rp[i]; q < a.rp[i + 1]; ++q) {
        const int j = a.ci[q];
        if ((forward ? j < i : j > i) && blk[j] != bi) succ[blk[j]].push_back(bi);
      }
    }
    for (int b = 0; b < nb; ++b) {
      std::sort(succ[b].begin(), succ[b].end());
      succ[b].erase(std::unique(succ[b].begin(), succ[b].end()), succ[b].end());
      for (int c : succ[b]) ++indeg[c];
    }
  }
  std::vector<int> order;
  order.reserve(nb);
  {
    auto prio = [&](int b) { return forward ? (int64_t)first[b] : -(int64_t)last[b]; };
    std::priority_queue<std::pair<int64_t, int>, std::vector<std::pair<int64_t, int>>, std::greater<>> ready;
    for (int b = 0; b < nb; ++b)
      if (indeg[b] == 0) ready.push({prio(b), b});
    while (!ready.empty()) {
      const int b = ready.top().second;
      ready.pop();
      order.push_back(b);
      for (int c : succ[b])
        if (--indeg[c] == 0) ready.push({prio(c), c});
    }
  }
  if ((int)order.size() != nb) return false;  // the blocks depend on each other in a cycle
  // rows of each block in (depth, row) order; slots and level boundaries
  std::vector<std::vector<int>> members(nb);
  for (int b = 0; b < nb; ++b) members[b].reserve(cnt[b]);
  for (int i = 0; i < n; ++i) members[blk[i]].push_back(i);
  s.nblk = nb;
  s.slot.assign(n, 0);
  s.block_of.assign(n, 0);
  s.blk_ptr.assign(nb + 1, 0);
  s.blk_lvl.assign(nb + 1, 0);
  s.rows.reserve(n);
  s.lvl_ptr.push_back(0);
  for (int t = 0; t < nb; ++t) {
    auto& m = members[order[t]];
    std::stable_sort(m.begin(), m.end(), [&](int x, int y) { return depth[x] < depth[y]; });
    s.blk_ptr[t] = (int)s.rows.size();
    s.blk_lvl[t] = (int)s.lvl_ptr.size() - 1;
    s.R = std::max(s.R, (int)m.size());
    for (size_t q = 0; q < m.size(); ++q) {
      const int i = m[q];
      if (q > 0 && depth[i] != depth[m[q - 1]]) s.lvl_ptr.push_back((int)s.rows.size());
      s.slot[i] = (int)q;
      s.block_of[i] = t;
      s.rows.push_back(i);
    }
    s.lvl_ptr.push_back((int)s.rows.size());
  }
  s.blk_ptr[nb] = (int)s.rows.size();
  s.blk_lvl[nb] = (int)s.lvl_ptr.size() - 1;
  return true;
}

void build_wave_schedule_parts(const HostCsr& a, bool forward, int W, int M, const std::vector<int>& parts,
                               int threads, WaveSchedule& s) {
  const int np = (int)parts.size() - 1;
  std::vector<WaveSchedule> ps(np);
  auto one = [&](int p) {
    const int r0 = parts[p], r1 = parts[p + 1];
    HostCsr sub;
    sub.n = sub.ncols = r1 - r0;
    sub.rp.resize(sub.n + 1);
    for (int i = r0; i <= r1; ++i) sub.rp[i - r0] = a.rp[i] - a.rp[r0];
    sub.ci.resize(sub.rp[sub.n]);
    for (int q = a.rp[r0]; q < a.rp[r1]; ++q) sub.ci[q - a.rp[r0]] = a.ci[q] - r0;
    const int stride = dominant_stride(sub);
    // a part whose segmented blocks would depend on each other in a cycle falls back
    // to contiguous blocks of the same number of rows
    if (!build_wave_schedule(sub, forward, W, M, stride, ps[p])) build_wave_schedule(sub, forward, W * M, 1, 0, ps[p]);
  };
  threads = std::max(1, std::min(threads, np));
  if (threads == 1) {
    for (int p = 0; p < np; ++p) one(p);
  } else {
    std::atomic<int> next{0};
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
      pool.emplace_back([&] {
        for (int p = next++; p < np; p = next++) one(p);
      });
    for (auto& th : pool) th.join();
  }
  if (np == 1) {
    s = std::move(ps[0]);
    s.blk_part.assign(s.nblk, 0);
    return;
  }
  // merge: each part's blocks keep their order; parts interleave by the fraction of
  // their blocks already placed
  std::vector<std::tuple<double, int, int>> key;  // (position, part, local block)
  for (int p = 0; p < np; ++p)
    for (int t = 0; t < ps[p].nblk; ++t) key.emplace_back((t + 0.5) / ps[p].nblk, p, t);
  std::stable_sort(key.begin(), key.end());
  s = WaveSchedule{};
  s.forward = forward;
  s.n = a.n;
  s.W = W;
  s.M = M;
  s.slot.assign(a.n, 0);
  s.block_of.assign(a.n, 0);
  s.blk_ptr.push_back(0);
  s.blk_lvl.push_back(0);
  s.lvl_ptr.push_back(0);
  s.rows.reserve(a.n);
  for (const auto& kt : key) {
    const int p = std::get<1>(kt), t = std::get<2>(kt);
    const WaveSchedule& q = ps[p];
    const int r0 = parts[p];
    const int tb = (int)s.blk_ptr.size() - 1;
    for (int m = q.blk_lvl[t]; m < q.blk_lvl[t + 1]; ++m) {
      for (int k = q.lvl_ptr[m]; k < q.lvl_ptr[m + 1]; ++k) {
        const int i = q.rows[k] + r0;
        s.rows.push_back(i);
        s.slot[i] = q.slot[q.rows[k]];
        s.block_of[i] = tb;
      }
      s.lvl_ptr.push_back((int)s.rows.size());
    }
    s.blk_ptr.push_back((int)s.rows.size());
    s.blk_lvl.push_back((int)s.lvl_ptr.size() - 1);
    s.blk_part.push_back(p);
    s.R = std::max(s.R, q.blk_ptr[t + 1] - q.blk_ptr[t]);
  }
  s.nblk = (int)s.blk_ptr.size() - 1;
  for (const auto& q : ps) {
    s.global_depth = std::max(s.global_depth, q.global_depth);
    s.stride = std::max(s.stride, q.stride);
  }
}

bool build_wave_pack(const HostCsr& a, const std::vector<double>& vals, const WaveSchedule& s,
                     const std::vector<std::pair<int, int>>& shapes, WavePack& w, int threads) {
  const int n = a.n;
  const bool fwd = s.forward;
  std::vector<int> part_max(std::max(1, threads), 0);
  std::atomic<int> slot_next{0};
  chunked(n, threads, 65536, [&](int64_t lo, int64_t hi) {
    int m = 0;
    for (int64_t i = lo; i < hi; ++i) {
      int c = 0;
      for (int q = a.rp[i]; q < a.rp[i + 1]; ++q) c += fwd ? (a.ci[q] < i) : (a.ci[q] > i);
      m = std::max(m, c);
    }
    part_max[slot_next++] = m;
  });
  const int maxlen = *std::max_element(part_max.begin(), part_max.end());
  const int nlev = (int)s.lvl_ptr.size() - 1;
  int tb = 0, K = 0;
  int64_t best = 0;
  for (const auto& sh : shapes) {
    if (sh.first * sh.second < maxlen || 64 % sh.first != 0) continue;
    const int G = 64 / sh.first;
    int64_t steps = 0;
    for (int m = 0; m < nlev; ++m) steps += (s.lvl_ptr[m + 1] - s.lvl_ptr[m] + G - 1) / G;
    if (tb == 0 || steps < best || (steps == best && sh.second < K)) {
      tb = sh.first;
      K = sh.second;
      best = steps;
    }
  }
  if (tb == 0) return false;
  const int G = 64 / tb;
  const size_t S = (size_t)best;
  w.tb = tb;
  w.k = K;
  w.nblk = s.nblk;
  w.R = s.R;
  w.nsteps = best;
  // first step of every block
  w.blk_step.assign(s.nblk + 1, 0);
  for (int t = 0; t < s.nblk; ++t) {
    int64_t c = 0;
    for (int m = s.blk_lvl[t]; m < s.blk_lvl[t + 1]; ++m) c += (s.lvl_ptr[m + 1] - s.lvl_ptr[m] + G - 1) / G;
    w.blk_step[t + 1] = w.blk_step[t] + (int)c;
  }
  w.row.resize(S * G);
  w.slot.resize(S * G);
  w.dinv.resize(S * G);
  w.col.resize(S * K * 64);
  w.val.resize(S * K * 64);
  // blocks fill disjoint step ranges: padding first, then the rows' entries
  chunked(s.nblk, threads, 4, [&](int64_t t0, int64_t t1) {
    for (int64_t t = t0; t < t1; ++t) {
      const size_t b0 = (size_t)w.blk_step[t], b1 = (size_t)w.blk_step[t + 1];
      std::fill(w.row.begin() + b0 * G, w.row.begin() + b1 * G, -1);
      std::fill(w.slot.begin() + b0 * G, w.slot.begin() + b1 * G, s.R);
      std::fill(w.dinv.begin() + b0 * G, w.dinv.begin() + b1 * G, 0.0);
      std::fill(w.col.begin() + b0 * K * 64, w.col.begin() + b1 * K * 64, s.R);
      std::fill(w.val.begin() + b0 * K * 64, w.val.begin() + b1 * K * 64, 0.0);
      size_t st = b0;
      for (int m = s.blk_lvl[t]; m < s.blk_lvl[t + 1]; ++m) {
        for (int p0 = s.lvl_ptr[m]; p0 < s.lvl_ptr[m + 1]; p0 += G, ++st) {
          const int p1 = std::min(p0 + G, s.lvl_ptr[m + 1]);
          for (int p = p0; p < p1; ++p) {
            const int gi = p - p0, i = s.rows[p];
            w.row[st * G + gi] = i;
            w.slot[st * G + gi] = s.slot[i];
            int e = 0;
            for (int q = a.rp[i]; q < a.rp[i + 1]; ++q) {
              const int j = a.ci[q];
              if (j == i) w.dinv[st * G + gi] = 1.0 / vals[q];
              if (!(fwd ? j < i : j > i)) continue;
              const size_t at = st * K * 64 + (size_t)(e / tb) * 64 + gi * tb + e % tb;
              w.col[at] = s.block_of[j] == t ? s.slot[j] : -(j + 1);
              w.val[at] = vals[q];
              ++e;
            }
          }
        }
      }
    }
  });
  return true;
}

int dense_spd_inverse(const HostCsr& a, std::vector<double>& inv, std::string* msg) {
  const int n = a.n;
  std::vector<double> g((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) g[(size_t)i * n + a.ci[p]] = a.v[p];
  // Cholesky A = G G^T (lower G), column by column
  for (int j = 0; j < n; ++j) {
    double d = g[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= g[(size_t)j * n + k] * g[(size_t)j * n + k];
    if (!(d > 0.0)) {
      if (msg) *msg = "coarsest matrix not positive definite at row " + std::to_string(j);
      return CPC_E_NOT_SPD;
    }
    d = std::sqrt(d);
    g[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = g[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= g[(size_t)i * n + k] * g[(size_t)j * n + k];
      g[(size_t)i * n + j] = s / d;
    }
  }
  // W = G^{-1} (lower triangular), then A^{-1} = W^T W
  std::vector<double> w((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    for (int i = c; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= g[(size_t)i * n + k] * w[(size_t)k * n + c];
      w[(size_t)i * n + c] = s / g[(size_t)i * n + i];
    }
  }
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int k = i; k < n; ++k) s += w[(size_t)k * n + i] * w[(size_t)k * n + j];
      inv[(size_t)i * n + j] = s;
      inv[(size_t)j * n + i] = s;
    }
  return CPC_OK;
}

}  // namespace cpc
