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
};
}  // namespace

// wr, wi: all n eigenvalues (descending real part); S (n x (nvec+1)): the
// wanted columns.  Returns the number of wanted columns, or -1 if the QR
// iteration failed.
extern "C" int ka_host_nonsym_eig(const double* H, int n, int nvec, double* wr, double* wi, double* S) {
  const int nv = std::min(nvec + 1, n);
  std::vector<double> work(ka::nonsym_work_doubles(n, nv)), v(n), w(n);
  ka::NsWork ws = ka::ns_work_split(work.data(), n, nv);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) ws.A[i + (size_t)j * n] = H[i + (size_t)j * n];
  HostTeam tm;
  ka::ns_hessenberg(tm, ws.A, n, n, ws.hsub, ws.beta, v.data(), w.data());
  ka::ns_band_fill(tm, ws.A, n, ws.hsub, n, ws.HB, ws.HT);
  if (ka::ns_qr_values(tm, ws.HB, n, ws.wr0, ws.wi0, ws.misc)) return -1;
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
