// Host build of the library's restart-basis stage (the same source the GPU
// kernel runs), for CPU unit tests of its logic.
#include <vector>

#include "../../paper_2101_00629_amd/csrc/basis_core.hpp"

namespace {
struct HostTeam {
  int tid() const { return 0; }
  int size() const { return 1; }
  void sync() const {}
  int argmax(double, int i) const { return i; }
};
}  // namespace

// G: n x n column-major.  W: n x n column-major (columns 0 .. r-1 written).
// Returns r.
extern "C" int ka_host_pchol_basis(const double* G, int n, double cut, double* W) {
  std::vector<double> work(ka::pchol_basis_work(n));
  HostTeam tm;
  return ka::pchol_basis(tm, G, n, n, cut, work.data(), W, n);
}
