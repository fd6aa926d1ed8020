// Resumable block Krylov eigensolver state (eigs.hip).
#pragma once
#include <chrono>
#include <cmath>
#include <vector>

#include "ka_internal.hpp"

namespace ka {

struct EigWork {
  double *X = nullptr, *AX = nullptr, *P = nullptr, *XS = nullptr, *AXS = nullptr, *R = nullptr, *T = nullptr;
  double *H = nullptr, *Hc = nullptr, *C = nullptr, *G = nullptr, *Rinv = nullptr, *theta = nullptr,
         *thetai = nullptr, *S = nullptr, *norms = nullptr, *ework = nullptr, *tnwork = nullptr,
         *nwork = nullptr, *Wm = nullptr, *Gm = nullptr, *pnorm = nullptr;
  int* status = nullptr;
};

// Device bytes of one solve's workspace (admission control of the server).
size_t eig_workspace_bytes(int64_t N, int M, int b);
// The problem's eigensolver workspace of at least `bytes`: its region's range
// (served requests), or a buffer kept between calls and replaced by a larger
// one only when a call needs more.
int eig_workspace(Problem* P, size_t bytes, char** out);

class EigRun {
 public:
  EigRun(Problem* P, int M, double tol, int maxit);
  ~EigRun();
  EigRun(const EigRun&) = delete;
  EigRun& operator=(const EigRun&) = delete;
  int start();                       // workspace, start block
  int pre_apply();                   // operator steps up to the kernel product of the pending block
  int post_apply(bool& done);        // the rest of the step; done = stop iterating
  int finish(double* lambda_host, double* V_dev, ka_info* info);
  size_t bytes() const { return cap_; }
  int matvecs() const { return matvecs_; }

 private:
  int alloc(size_t bytes, double** out);
  int orth_block(int k, int pw);
  int rayleigh_ritz(bool& stop);
  double modulus(int i) const { return sym_ ? std::fabs(th_[i]) : std::hypot(th_[i], thi_[i]); }

  Problem* P_;
  hipStream_t s_;
  int M_;
  double tol_;
  int maxit_;
  bool verbose_ = false;
  bool sym_ = true;
  double noise_ = 0.0;
  int nev_ = 0, m_max_ = 0;
  bool full_ = false;
  EigWork w_;
  char* base_ = nullptr;   // workspace of this solve (owned by the problem), bump-allocated
  size_t cap_ = 0, off_ = 0;
  uint64_t rng_counter_ = 0;
  int k_ = 0, pw_ = 0, cycles_ = 0, matvecs_ = 0, nconv_ = 0, Meff_ = 0, nret_ = 0, stall_ = 0, floor_ok_ = 0;
  double max_res_ = 0.0, max_imag_ = 0.0, best_res_ = 1e300, pairs0_ = 0.0;
  bool converged_ = false;
  std::vector<double> th_, thi_, rn_;
  std::vector<double> th_prev_, thi_prev_;   // non-symmetric: Ritz values of the previous Rayleigh-Ritz step
  std::chrono::steady_clock::time_point t_start_;
};

}  // namespace ka
