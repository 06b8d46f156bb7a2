// Host-only entry points over the library's SETUP code (host_setup.cpp), built into
// libcpc_host.so so that tests can check the coarsening, interpolation, ILU(0) and
// sweep schedules on a machine without a GPU. Not part of the solver's C-ABI.
#include <cstring>
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

int cpch_dense_inverse(int n, const int* rp, const int* ci, const double* v, double* inv) {
  HostCsr a = make_csr(n, rp, ci, v);
  std::vector<double> out;
  int st = cpc::dense_spd_inverse(a, out, nullptr);
  if (st == 0) std::memcpy(inv, out.data(), sizeof(double) * out.size());
  return st;
}

}  // extern "C"
