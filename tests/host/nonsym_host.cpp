// Host build of the library's small non-symmetric eigensolve core (the same
// source the GPU wave runs), for CPU unit tests of its logic.
#include <vector>

#include "../../paper_2101_00629_amd/csrc/nonsym_core.hpp"

namespace {
struct HostTeam {
  double* scratch;
  int tid() const { return 0; }
  int size() const { return 1; }
  void sync() const {}
  double sum(double x) const { return x; }
};
}  // namespace

extern "C" int ka_host_nonsym_eig(const double* H, int n, double* wr, double* wi, double* S) {
  std::vector<double> work(ka::nonsym_work_doubles(n)), scratch(6 * n + 6);
  HostTeam tm{scratch.data()};
  int status = -1;
  ka::nonsym_core(tm, H, n, n, wr, wi, S, n, work.data(), &status);
  return status;
}
