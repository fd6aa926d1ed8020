// Host build of the library's small non-symmetric eigensolve stages (the same
// source the GPU kernels run), for CPU unit tests of their logic.
#include <algorithm>
#include <cmath>
#include <vector>

#include "../../paper_2101_00629_amd/csrc/nonsym_core.hpp"

namespace {
struct HostTeam {
  int tid() const { return 0; }
  int size() const { return 1; }
  void sync() const {}
  double sum(double x) const { return x; }
  int imax(int x) const { return x; }
  int gsize() const { return 1; }
  int group() const { return 0; }
  void gsync() const {}
  double gpick(double v, int) const { return v; }
};

// eigenvalues of the trailing block for the multishift sweeps
struct HostSmallEig {
  int operator()(double* sb, int ns, double* sr, double* si, double tol) const {
    HostTeam tm;
    return ka::ns_qr_values(tm, sb, ns, sr, si, nullptr, tol);
  }
};

// eigenvalue stage: the double-shift loop (ms == 0) or the multishift driver;
// fast_n > 0 also moves the band to a second buffer of that order once the
// leading block fits, as the device does with LDS
int qr_values(ka::NsWork& ws, int n, int ms, int fast_n) {
  HostTeam tm;
  if (!ms) return ka::ns_qr_values(tm, ws.HB, n, ws.wr0, ws.wi0, ws.misc);
  std::vector<double> scr(ka::ns_ms_scratch_doubles()), fast(fast_n > 0 ? ka::ns_band_doubles(fast_n) : 0);
  return ka::ns_qr_values_ms(tm, ws.HB, n, ws.wr0, ws.wi0, ws.misc, scr.data(), HostSmallEig(),
                             fast_n > 0 ? fast.data() : nullptr, fast_n);
}
}  // namespace

// wr, wi: all n eigenvalues (descending real part); S (n x (nvec+1)): the
// wanted columns.  Returns the number of wanted columns, or -1 if the QR
// iteration failed.
extern "C" int ka_host_nonsym_eig_ms(const double* H, int n, int nvec, double* wr, double* wi, double* S, int ms,
                                     int fast_n) {
  const int nv = std::min(nvec + 1, n);
  std::vector<double> work(ka::nonsym_work_doubles(n, nv)), v(n), w(n);
  ka::NsWork ws = ka::ns_work_split(work.data(), n, nv);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) ws.A[i + (size_t)j * n] = H[i + (size_t)j * n];
  HostTeam tm;
  ka::ns_hessenberg(tm, ws.A, n, n, ws.hsub, ws.beta, v.data(), w.data());
  ka::ns_band_fill(tm, ws.A, n, ws.hsub, n, ws.HB, ws.HT);
  if (qr_values(ws, n, ms, fast_n)) return -1;
  for (int c = 0; c < n; ++c) {
    const int r = ka::ns_rank(ws.wr0, n, c);
    ws.wr[r] = ws.wr0[c];
    ws.wi[r] = ws.wi0[c];
  }
  const int nw = ka::ns_wanted(ws.wi, n, nvec);
  const double scale = ka::ns_scale(ws.wr, ws.wi, n);
  std::vector<double> Ur(ka::ns_lu_plane(n)), Ui(ka::ns_lu_plane(n)), ml(3 * n), xs(2 * n);
  for (int c = 0; c < nw; ++c)
    if (ka::ns_is_entry(ws.wi, c) && ka::ns_cluster_first(ws.wr, ws.wi, c, ka::kNsClusterGap * scale))
      ka::ns_invit_team(tm, ws.HT, ws.hsub, n, ws.wr, ws.wi, c, nw, nv, scale, ws.V, Ur.data(), Ui.data(), ml.data(),
                        xs.data());
  for (int c = 0; c < nw; ++c) ka::sym_back_transform(ws.A, ws.beta, n, ws.V + c, nv);
  for (int c = 0; c < n; ++c) {
    wr[c] = ws.wr[c];
    wi[c] = ws.wi[c];
  }
  for (int c = 0; c < nw; ++c) {
    const int c0 = ka::ns_is_entry(ws.wi, c) ? c : c - 1;
    const bool pair = ws.wi[c0] > 0.0;
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      s += ws.V[(size_t)i * nv + c0] * ws.V[(size_t)i * nv + c0];
      if (pair) s += ws.V[(size_t)i * nv + c0 + 1] * ws.V[(size_t)i * nv + c0 + 1];
    }
    const double sc = s > 0.0 ? 1.0 / std::sqrt(s) : 0.0;
    for (int i = 0; i < n; ++i) S[i + (size_t)c * n] = ws.V[(size_t)i * nv + c] * sc;
  }
  return nw;
}

extern "C" int ka_host_nonsym_eig(const double* H, int n, int nvec, double* wr, double* wi, double* S) {
  return ka_host_nonsym_eig_ms(H, n, nvec, wr, wi, S, 0, 0);
}

// eigenvalues only, in the order the QR stage finds them; returns the QR
// stage's status (0, or 1 when an eigenvalue took too many iterations)
extern "C" int ka_host_nonsym_values(const double* H, int n, double* wr, double* wi, int ms, int fast_n) {
  std::vector<double> work(ka::nonsym_work_doubles(n, 1)), v(n), w(n);
  ka::NsWork ws = ka::ns_work_split(work.data(), n, 1);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) ws.A[i + (size_t)j * n] = H[i + (size_t)j * n];
  HostTeam tm;
  ka::ns_hessenberg(tm, ws.A, n, n, ws.hsub, ws.beta, v.data(), w.data());
  ka::ns_band_fill(tm, ws.A, n, ws.hsub, n, ws.HB, nullptr);
  const int rc = qr_values(ws, n, ms, fast_n);
  for (int c = 0; c < n; ++c) {
    wr[c] = ws.wr0[c];
    wi[c] = ws.wi0[c];
  }
  return rc;
}

// first column of (H - s1 I)(H - s2 I), rows 0..2, for an upper Hessenberg H
// (column-major, n >= 3), as the multishift sweep introduces a bulge
extern "C" void ka_host_ms_first_column(const double* H, int n, double sr1, double si1, double sr2, double si2,
                                        double* v) {
  std::vector<double> hb(ka::ns_band_doubles(n), 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j + 1 && i < n; ++i) hb[ka::ns_band_index(i, j)] = H[i + (size_t)j * n];
  ka::ns_ms_first_column(ka::NsBand{hb.data()}, 0, sr1, si1, sr2, si2, v);
}

// the multishift sweep's pairing of shifts, in place
extern "C" void ka_host_pair_shifts(double* sr, double* si, int ns) { ka::ns_pair_shifts(sr, si, ns); }
