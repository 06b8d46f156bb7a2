// Host-only entry points over the library's SETUP code (host_setup.cpp), built into
// libcpc_host.so so that tests can check the coarsening, interpolation, ILU(0) and
// sweep schedules on a machine without a GPU. Not part of the solver's C-ABI.
#include <algorithm>
#include <cstring>
#include <utility>
#include <vector>

#include "host_setup.hpp"

using cpc::HostCsr;

static HostCsr make_csr(int n, const int* rp, const int* ci, const double* v) {
  HostCsr a;
  a.n = n;
  a.ncols = n;
  a.rp.assign(rp, rp + n + 1);
  a.ci.assign(ci, ci + rp[n]);
  a.v.assign(v, v + rp[n]);
  return a;
}

extern "C" {

int cpch_ilu0(int n, const int* rp, const int* ci, const double* v, double* lu) {
  HostCsr a = make_csr(n, rp, ci, v);
  std::vector<double> out;
  int st = cpc::ilu0_factor(a, out, nullptr);
  std::memcpy(lu, out.data(), sizeof(double) * out.size());
  return st;
}

// ILU(k): call with f_rp only to get nnz (returned, or -status), then with all arrays.
long cpch_iluk(int n, const int* rp, const int* ci, const double* v, int k, int* f_rp, int* f_ci, double* f_v,
               int* f_lev) {
  HostCsr a = make_csr(n, rp, ci, v);
  HostCsr f;
  std::vector<int> lev;
  int st = cpc::iluk_factor(a, k, f, lev, nullptr);
  if (st) return -st;
  if (f_rp) std::memcpy(f_rp, f.rp.data(), sizeof(int) * (n + 1));
  if (f_ci) std::memcpy(f_ci, f.ci.data(), sizeof(int) * f.ci.size());
  if (f_v) std::memcpy(f_v, f.v.data(), sizeof(double) * f.v.size());
  if (f_lev) std::memcpy(f_lev, lev.data(), sizeof(int) * lev.size());
  return (long)f.ci.size();
}

int cpch_rs_coarsen(int n, const int* rp, const int* ci, const double* v, double theta, int* cf) {
  HostCsr a = make_csr(n, rp, ci, v);
  std::vector<int> c;
  int nc = cpc::rs_coarsen(a, theta, c);
  std::memcpy(cf, c.data(), sizeof(int) * n);
  return nc;
}

// P for a given splitting; call with p_rp only to get nnz (returned), then with all arrays.
long cpch_rs_interp(int n, const int* rp, const int* ci, const double* v, double theta, const int* cf, int* p_rp,
                    int* p_ci, double* p_v) {
  HostCsr a = make_csr(n, rp, ci, v);
  std::vector<int> c(cf, cf + n);
  int nc = 0;
  for (int i = 0; i < n; ++i) nc += (cf[i] == 1);
  HostCsr P;
  cpc::rs_interpolation(a, theta, c, nc, P);
  if (p_rp) std::memcpy(p_rp, P.rp.data(), sizeof(int) * (n + 1));
  if (p_ci) std::memcpy(p_ci, P.ci.data(), sizeof(int) * P.nnz());
  if (p_v) std::memcpy(p_v, P.v.data(), sizeof(double) * P.nnz());
  return (long)P.nnz();
}

// Sweep schedule: sizes[0..6] = nblk, nlev_total, nwait, global_depth, max_local_levels, R,
// max_level_entries. Arrays may be null on a first call that only asks for sizes.
int cpch_sweep(int n, const int* rp, const int* ci, const double* v, int forward, int R, int max_entries,
               int* sizes, int* perm,
               int* blk_beg, int* blk_end, int* lvl_ptr, int* wait_ptr, int* wait_blk, int* wait_need, int* publish,
               int* blk_row) {
  HostCsr a = make_csr(n, rp, ci, v);
  cpc::SweepSchedule s = cpc::build_sweep(a, forward != 0, R, max_entries);
  const int nl = (int)s.lvl_ptr.size() - 1;
  sizes[0] = s.nblk;
  sizes[1] = nl;
  sizes[2] = (int)s.wait_blk.size();
  sizes[3] = s.global_depth;
  sizes[4] = s.max_local_levels;
  sizes[5] = s.R;
  sizes[6] = (int)s.max_level_entries;
  if (perm) std::memcpy(perm, s.perm.data(), sizeof(int) * s.perm.size());
  if (blk_beg) std::memcpy(blk_beg, s.blk_beg.data(), sizeof(int) * s.nblk);
  if (blk_end) std::memcpy(blk_end, s.blk_end.data(), sizeof(int) * s.nblk);
  if (lvl_ptr) std::memcpy(lvl_ptr, s.lvl_ptr.data(), sizeof(int) * (nl + 1));
  if (wait_ptr) std::memcpy(wait_ptr, s.wait_ptr.data(), sizeof(int) * (nl + 1));
  if (wait_blk) std::memcpy(wait_blk, s.wait_blk.data(), sizeof(int) * s.wait_blk.size());
  if (wait_need) std::memcpy(wait_need, s.wait_need.data(), sizeof(int) * s.wait_need.size());
  if (publish) std::memcpy(publish, s.publish.data(), sizeof(int) * nl);
  if (blk_row) std::memcpy(blk_row, s.blk_row.data(), sizeof(int) * (s.nblk + 1));
  return 0;
}

// Sequential emulation of the one-wave sweep kernel on its pack: blocks in ticket
// order, the steps of a block in order including the padding steps the kernel's ring
// of `ring` steps runs past the end, every load addressed as the kernel addresses it
// (the entry data of the step `ring` ahead, clamped to the block's last step). The
// schedule has blocks of W-row segments, M per block, spaced by the matrix's dominant
// coupling distance (M = 1: contiguous blocks of W rows). Returns 0 with
// x = T^{-1} f (T = D+L forward, D+U backward; unit diagonal when unit != 0) and
// shape = {tb, k, nblk, nsteps, R, M, stride}, or a negative code: -1 an address outside
// its array, -2 a value of the block's own rows read before it was written, -3 a value
// of another block read before that block wrote it, -4 a row written twice, into a slot
// taken by another row, or never, -5 no pack (a row longer than every shape), -6 the
// blocks' dependency graph has a cycle.
// Block starts of the four-wave sweep schedule with R rows per block, no block spanning
// two of the parts (parts: nparts + 1 boundaries, or null). Writes at most cap starts
// (the last one = n) and returns their number.
int cpch_block_starts(int n, const int* rp, const int* ci, const double* v, int R, const int* parts, int nparts,
                      int* out, int cap) {
  HostCsr a = make_csr(n, rp, ci, v);
  std::vector<int> pv;
  if (parts && nparts > 0) pv.assign(parts, parts + nparts + 1);
  const std::vector<int> st = cpc::sweep_block_starts(a, R, pv.empty() ? nullptr : &pv);
  for (int i = 0; i < (int)st.size() && i < cap; ++i) out[i] = st[i];
  return (int)st.size();
}

int cpch_wave_emulate(int n, const int* rp, const int* ci, const double* v, int forward, int W, int M, int unit,
                      int ring, const double* f, double* x, int* shape, const int* parts, int nparts) {
  HostCsr a = make_csr(n, rp, ci, v);
  int stride = cpc::dominant_stride(a);
  cpc::WaveSchedule s;
  if (parts && nparts > 0) {  // per-system schedules of a block-diagonal matrix
    cpc::build_wave_schedule_parts(a, forward != 0, W, M, std::vector<int>(parts, parts + nparts + 1), 4, s);
    stride = s.stride;
  } else if (!cpc::build_wave_schedule(a, forward != 0, W, M, stride, s)) {
    return -6;
  }
  std::vector<std::pair<int, int>> shapes;
  for (int tb : {1, 2, 4, 8, 16})
    for (int k : {2, 4}) shapes.push_back({tb, k});
  cpc::WavePack w;
  if (!cpc::build_wave_pack(a, a.v, s, shapes, w, 3)) return -5;
  const int K = w.k, TB = w.tb, G = 64 / TB;
  shape[0] = TB;
  shape[1] = K;
  shape[2] = w.nblk;
  shape[3] = (int)w.nsteps;
  shape[4] = w.R;
  shape[5] = s.M;
  shape[6] = stride;
  std::vector<char> xw(n, 0);
  std::vector<double> xs(w.R + 1, 0.0);
  std::vector<int> owner(w.R + 1, -1);
  const size_t ncol = w.col.size(), nrow = w.row.size();
  if ((int)w.blk_step.size() != w.nblk + 1 || w.blk_step[w.nblk] != w.nsteps) return -1;
  for (int t = 0; t < w.nblk; ++t) {
    const int s0 = w.blk_step[t], s1 = w.blk_step[t + 1];
    if (!(s1 > s0)) return -1;
    std::fill(owner.begin(), owner.end(), -1);
    owner[w.R] = n;  // the zero slot
    xs[w.R] = 0.0;
    const int last = s0 + ((s1 - s0 + ring - 1) / ring) * ring;  // steps the ring runs
    for (int st = s0; st < last + ring; ++st) {
      // every step the kernel issues loads for, clamped as the kernel clamps them
      const int sc = st < s1 ? st : s1 - 1;
      for (int lane = 0; lane < 64; ++lane)
        for (int k = 0; k < K; ++k)
          if ((size_t)sc * K * 64 + (size_t)k * 64 + lane >= ncol) return -1;
      for (int g = 0; g < G; ++g)
        if ((size_t)sc * G + g >= nrow) return -1;
      if (st >= last) continue;  // loads issued by the last steps, never computed
      const bool valid = st < s1;
      for (int g = 0; g < G; ++g) {
        const int row = valid ? w.row[(size_t)sc * G + g] : -1;
        const int sl = w.slot[(size_t)sc * G + g];
        if (sl < 0 || sl > w.R) return -1;
        double sum = 0.0;
        for (int l = 0; l < TB; ++l) {
          const int lane = g * TB + l;
          for (int k = 0; k < K; ++k) {
            const size_t at = (size_t)sc * K * 64 + (size_t)k * 64 + lane;
            const int c = w.col[at];
            double xv;
            if (c >= 0) {
              if (c > w.R) return -1;
              if (owner[c] < 0) return -2;
              xv = xs[c];
            } else {
              const int j = -(c + 1);
              if (j < 0 || j >= n) return -1;
              if (!xw[j]) return -3;
              xv = x[j];
            }
            sum += w.val[at] * xv;
          }
        }
        if (row < 0) continue;
        if (row >= n || xw[row] || sl >= w.R || owner[sl] >= 0) return -4;
        const double xi = unit ? f[row] - sum : (f[row] - sum) * w.dinv[(size_t)sc * G + g];
        xs[sl] = xi;
        owner[sl] = row;
        x[row] = xi;
        xw[row] = 1;
      }
    }
  }
  for (int i = 0; i < n; ++i)
    if (!xw[i]) return -4;
  return 0;
}

int cpch_dense_inverse(int n, const int* rp, const int* ci, const double* v, double* inv) {
  HostCsr a = make_csr(n, rp, ci, v);
  std::vector<double> out;
  int st = cpc::dense_spd_inverse(a, out, nullptr);
  if (st == 0) std::memcpy(inv, out.data(), sizeof(double) * out.size());
  return st;
}

}  // extern "C"
