// Host build of the library's small symmetric eigensolve stages (the same
// source the GPU kernels run), for CPU unit tests of their logic.
#include <vector>

#include "../../paper_2101_00629_amd/csrc/sym_core.hpp"

namespace {
struct HostTeam {
  int tid() const { return 0; }
  int size() const { return 1; }
  void sync() const {}
  double sum(double x) const { return x; }
  void sumv(const double* x, int k, double* out) const {
    for (int i = 0; i < k; ++i) out[i] = x[i];
  }
};
}  // namespace

// theta descending (all n), S (n x nvec column-major) the unit eigenvectors of
// the nvec largest; returns the number of clusters met among them.  nb > 0
// takes the blocked tridiagonalisation with panels of nb columns.
extern "C" int ka_host_sym_eig_nb(const double* H, int n, int nvec, double* theta, double* S, int nb) {
  std::vector<double> work(ka::sym_tri_work_doubles(n)), v(n), w(n);
  ka::SymWork sw = ka::sym_work_split(work.data(), n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) sw.A[i + (size_t)j * n] = 0.5 * (H[i + (size_t)j * n] + H[j + (size_t)i * n]);
  HostTeam tm;
  if (nb > 0) {
    std::vector<double> V((size_t)n * ka::kSymNbMax), W((size_t)n * ka::kSymNbMax), yz(2 * ka::kSymNbMax);
    ka::sym_tridiagonalize_blocked(tm, sw.A, n, sw.d, sw.e, sw.beta, v.data(), w.data(), V.data(), W.data(),
                                   yz.data(), nb);
  } else {
    ka::sym_tridiagonalize(tm, sw.A, n, sw.d, sw.e, sw.beta, v.data(), w.data());
  }
  ka::sym_bounds(sw.d, sw.e, n, sw.bnd);
  const double pivmin = ka::sym_pivmin(sw.bnd);
  for (int k = 0; k < n; ++k) {
    // one wave of 64 lanes, emulated
    double lo = sw.bnd[0], hi = sw.bnd[1];
    for (int r = 0; r < ka::kSymSectionRounds && !ka::sym_section_done(lo, hi, sw.bnd); ++r) {
      uint64_t mask = 0;
      for (int t = 0; t < 64; ++t)
        if (ka::sym_sturm_count(sw.d, sw.e, n, ka::sym_section_point(lo, hi, t, 64), pivmin) > k)
          mask |= 1ull << t;
      ka::sym_section_narrow(lo, hi, mask, 64);
    }
    sw.lam[k] = 0.5 * (lo + hi);
  }
  int clusters = 0;
  std::vector<double> xw(n), fw(5 * (size_t)n);
  for (int k = n - 1; k >= n - nvec; --k)
    if (ka::sym_cluster_top(sw.lam, n, k, sw.bnd)) {
      ++clusters;
      ka::sym_inverse_iteration(sw.d, sw.e, n, sw.lam, k, n - nvec, sw.bnd, sw.V, fw.data(), (size_t)n, 1, xw.data(),
                                1);
    }
  for (int k = n - nvec; k < n; ++k) ka::sym_back_transform(sw.A, sw.beta, n, sw.V + k, n);
  for (int k = 0; k < n; ++k) theta[k] = sw.lam[n - 1 - k];
  for (int k = 0; k < nvec; ++k) {
    const int src = n - 1 - k;
    for (int i = 0; i < n; ++i) S[i + (size_t)k * n] = sw.V[(size_t)i * n + src];
  }
  return clusters;
}

extern "C" int ka_host_sym_eig(const double* H, int n, int nvec, double* theta, double* S) {
  return ka_host_sym_eig_nb(H, n, nvec, theta, S, 0);
}
