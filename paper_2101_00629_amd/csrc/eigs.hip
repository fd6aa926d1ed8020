// Block Krylov eigensolver with thick restarts for the standard-form operator
// A' (paper Sec. 3, eq. standard; the paper's "iterative eigenvalue solver"
// is not named, this is the reading used here).
//
// State on the device, FP64:  X (N x m) orthonormal basis, AX = A' X,
// H = X^T A' X, a pending block P orthonormal to X.  One cycle:
//   append P to X, AP = A' P (one block application of A'), update H,
//   P <- orth(AP - X X^T AP)  (block classical Gram-Schmidt twice, then
//   Cholesky-QR twice; a rank-deficient block is replaced by fresh random
//   vectors), and when X is full: Rayleigh-Ritz (small dense eigensolve of H),
//   residuals |A'y - theta y|, convergence test, thick restart keeping the
//   leading nev Ritz vectors.
// Galerkin (symmetric A'): tridiagonal route on H (Householder, multisection,
// inverse iteration), X <- X S, H <- diag(theta).
// Collocation (A' = Z^-1 A, non-symmetric): Hessenberg QR on H, restart onto
// an orthonormal basis of the wanted Ritz vectors (W from a pivoted Cholesky of
// their Gram matrix, twice), H <- W^T S^T H S W.
//
// The solve is a resumable state machine (EigRun): pre_apply() issues the
// operator steps up to the kernel product, the caller runs the product
// (alone, or batched with other problems), post_apply() finishes the step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "eigrun.hpp"

namespace ka {

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(KA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define KA_TRY(expr)               \
  do {                             \
    int r_ = (expr);               \
    if (r_ != KA_OK) return r_;    \
  } while (0)

namespace {

__global__ void mirror_kernel(double* H, int ld, int k, int pw) {
  // H[k + j][i] = H[i][k + j] for i < k, j < pw  (column-major: (r, c) at r + c ld)
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= k * pw) return;
  const int i = id % k, j = id / k;
  H[(k + j) + (int64_t)i * ld] = H[i + (int64_t)(k + j) * ld];
}

__global__ void set_diag_kernel(double* H, int ld, int n, const double* theta) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * n) return;
  const int i = id % n, j = id / n;
  H[i + (int64_t)j * ld] = (i == j) ? theta[i] : 0.0;
}

__global__ void symmetrize_block_kernel(double* H, int ld, int k, int pw) {
  // average the new diagonal block (k..k+pw) with its transpose
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= pw * pw) return;
  const int i = id % pw, j = id / pw;
  if (i >= j) return;
  double* a = H + (k + i) + (int64_t)(k + j) * ld;
  double* b = H + (k + j) + (int64_t)(k + i) * ld;
  const double v = 0.5 * (*a + *b);
  *a = v;
  *b = v;
}

}  // namespace

// Rank cut of the restart basis: a kept Ritz vector whose squared distance
// from the span of the ones chosen before it is at or below this fraction of
// the largest squared norm is dropped (the vectors are normalised).
constexpr double kBasisCut = 1e-12;

// ---- sizes ----------------------------------------------------------------
static void basis_sizes(int64_t N, int M, int b, int& nev, int& m_max, bool& full) {
  nev = (int)std::min<int64_t>(N, (int64_t)M + b);
  const int nb = std::max(2, (nev + 2 * b - 1) / (2 * b));
  m_max = nev + nb * b;
  full = false;
  if ((int64_t)m_max >= N) {   // small problem: the Krylov space becomes the whole space
    m_max = (int)N;
    full = true;
  }
}

static size_t tn_work_doubles(int m_max, int b, int64_t N) {
  size_t tnw = (size_t)m_max * m_max;
  for (int m = 1; m <= m_max; ++m) {
    tnw = std::max(tnw, dgemm_tn_work(m, b, N));
    tnw = std::max(tnw, dgemm_tn_work(b, m, N));
  }
  return tnw;
}

size_t eig_workspace_bytes(int64_t N, int M, int b) {
  int nev, m_max;
  bool full;
  basis_sizes(N, M, b, nev, m_max, full);
  const int ncol = nev + 1;
  auto al = [](size_t x) { return (x + 255) / 256 * 256 + 256; };
  size_t s = 0;
  s += 2 * al((size_t)N * m_max * 8);
  s += al((size_t)N * b * 8);
  s += al((size_t)N * std::max(ncol, b) * 8);
  s += 3 * al((size_t)N * ncol * 8);
  s += 5 * al((size_t)m_max * m_max * 8);
  s += al((size_t)m_max * b * 8) + 2 * al((size_t)b * b * 8) + 3 * al((size_t)m_max * 8);
  s += al(std::max({basis_work(m_max), sym_tri_work(m_max), nonsym_eig_work(m_max, std::min(nev + 1, m_max))}) * 8);
  s += al(tn_work_doubles(m_max, b, N) * 8);
  s += al(column_norms_work(N, std::max(ncol, b)) * 8) + al((size_t)b * 8) + al(256);
  return s;
}

// ---- EigRun -----------------------------------------------------------------
EigRun::EigRun(Problem* P, int M, double tol, int maxit) : P_(P), s_(P->stream), M_(M), tol_(tol), maxit_(maxit) {
  const char* v = std::getenv("KA_VERBOSE");
  verbose_ = v && v[0] && v[0] != '0';
}

EigRun::~EigRun() = default;   // the workspace belongs to the problem

int eig_workspace(Problem* P, size_t bytes, char** out) {
  if (P->region.base) {
    // served request: carved once from its range (sized by ka_request_bytes)
    if (!P->eig_buf) {
      if (P->region.used + bytes > P->region.size) return fail(KA_ERR_OOM, "eigensolver workspace exceeds the request's memory");
      P->eig_buf = P->region.base + P->region.used;
      P->region.used += bytes;
      P->eig_buf_bytes = bytes;
    } else if (P->eig_buf_bytes < bytes) {
      return fail(KA_ERR_OOM, "eigensolver workspace exceeds the request's memory");
    }
  } else if (P->eig_buf_bytes < bytes) {
    if (P->eig_buf) {
      // earlier solves on this stream may still read the old buffer
      if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(KA_ERR_HIP, "stream synchronize failed");
      (void)hipFree(P->eig_buf);
      P->eig_buf = nullptr;
      P->eig_buf_bytes = 0;
    }
    if (hipMalloc(&P->eig_buf, bytes) != hipSuccess) {
      P->eig_buf = nullptr;
      return fail(KA_ERR_OOM, "eigensolver workspace allocation failed");
    }
    P->eig_buf_bytes = bytes;
  }
  *out = (char*)P->eig_buf;
  return KA_OK;
}

int EigRun::alloc(size_t bytes, double** out) {
  bytes = (bytes + 255) / 256 * 256;
  if (bytes == 0) bytes = 256;
  if (off_ + bytes > cap_) return fail(KA_ERR_OOM, "eigensolver workspace layout exceeds its size");
  *out = (double*)(base_ + off_);
  off_ += bytes;
  return KA_OK;
}

int64_t lambda_doubles(const ka_desc& d, int M) { return d.method == KA_COLLOCATION ? 2 * (int64_t)M : M; }

// Orthonormalise P (N x pw) against X[:, :k] (block CGS twice) and within
// itself (Cholesky-QR twice).  Rank-deficient blocks are redrawn at random:
// a column is rank-deficient when what is left of it after the projections
// is below kOrthKeep of its norm before them (the Krylov space is exhausted
// along it, and the rest is rounding, which normalisation would blow up into
// directions not orthogonal to X), or when the Cholesky factorisation of the
// block's Gram matrix loses a pivot.
int EigRun::orth_block(int k, int pw) {
  const int64_t N = P_->N;
  for (int attempt = 0; attempt < 4; ++attempt) {
    if (k > 0) {
      HIP_TRY(column_norms(w_.P, N, pw, N, w_.pnorm, w_.nwork, s_));
      for (int pass = 0; pass < 2; ++pass) {
        HIP_TRY(dgemm_tn(k, pw, N, 1.0, w_.X, N, w_.P, N, 0.0, w_.C, k, w_.tnwork, s_));
        HIP_TRY(dgemm_nn(N, pw, k, -1.0, w_.X, N, w_.C, k, 1.0, w_.P, N, s_));
      }
    }
    // both passes run before the one host read of their two status words (a
    // block that fails the first pass is redrawn all the same)
    for (int pass = 0; pass < 2; ++pass) {
      HIP_TRY(dgemm_tn(pw, pw, N, 1.0, w_.P, N, w_.P, N, 0.0, w_.G, pw, w_.tnwork, s_));
      HIP_TRY(chol_upper_inv(w_.G, pw, pw, w_.Rinv, pw, w_.status + pass, s_,
                             pass == 0 && k > 0 ? w_.pnorm : nullptr));
      HIP_TRY(dgemm_nn(N, pw, pw, 1.0, w_.P, N, w_.Rinv, pw, 0.0, w_.T, N, s_));
      HIP_TRY(copy_cols(w_.T, N, w_.P, N, N, pw, s_));
    }
    int st[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(st, w_.status, sizeof(st), hipMemcpyDeviceToHost, s_));
    HIP_TRY(hipStreamSynchronize(s_));
    if (!st[0] && !st[1]) return KA_OK;
    // Krylov space exhausted along some direction: continue with random ones
    HIP_TRY(fill_normal(w_.P, N, pw, N, P_->d.seed, ++rng_counter_, s_));
  }
  return fail(KA_ERR_SINGULAR, "could not extend the Krylov basis");
}

int EigRun::start() {
  t_start_ = std::chrono::steady_clock::now();
  sym_ = P_->d.method != KA_COLLOCATION;
  const int64_t N = P_->N;
  const int b = P_->b;
  if (M_ < 1 || M_ > N) return fail(KA_ERR_ARG, "M must be in 1..N");
  if (!(tol_ > 0)) tol_ = 1e-6;
  if (maxit_ <= 0) maxit_ = 100;
  // Residuals of an operator applied in FP32 (or split BF16) cannot fall
  // below a few units of its rounding times |theta_1|; below that level the
  // Ritz values no longer move.  Symmetric problems tolerate this (eigenvalue
  // error ~ r^2 / gap); for the non-symmetric collocation operator the error
  // is first order in r, so its floor is set 20x lower, close to what the
  // FP32 operator can resolve.
  if (sym_) noise_ = P_->d.precision == KA_FP32 ? 4e-6 : 1e-4;
  else noise_ = P_->d.precision == KA_FP32 ? 2e-7 : 5e-6;
  basis_sizes(N, M_, b, nev_, m_max_, full_);
  if (m_max_ > 1000) return fail(KA_ERR_ARG, "M too large for the dense Rayleigh-Ritz (M + block <= ~600)");
  const int ncol = nev_ + 1;   // room for a complex pair that straddles nev
  const int m = m_max_;
  cap_ = eig_workspace_bytes(N, M_, b);
  off_ = 0;
  KA_TRY(eig_workspace(P_, cap_, &base_));
  KA_TRY(alloc((size_t)N * m * 8, &w_.X));
  KA_TRY(alloc((size_t)N * m * 8, &w_.AX));
  KA_TRY(alloc((size_t)N * b * 8, &w_.P));
  KA_TRY(alloc((size_t)N * std::max(ncol, b) * 8, &w_.T));
  KA_TRY(alloc((size_t)N * ncol * 8, &w_.XS));
  KA_TRY(alloc((size_t)N * ncol * 8, &w_.AXS));
  KA_TRY(alloc((size_t)N * ncol * 8, &w_.R));
  KA_TRY(alloc((size_t)m * m * 8, &w_.H));
  KA_TRY(alloc((size_t)m * m * 8, &w_.Hc));
  KA_TRY(alloc((size_t)m * m * 8, &w_.Wm));
  KA_TRY(alloc((size_t)m * m * 8, &w_.Gm));
  KA_TRY(alloc((size_t)m * m * 8, &w_.S));
  KA_TRY(alloc((size_t)m * b * 8, &w_.C));
  KA_TRY(alloc((size_t)b * b * 8, &w_.G));
  KA_TRY(alloc((size_t)b * b * 8, &w_.Rinv));
  KA_TRY(alloc((size_t)m * 8, &w_.theta));
  KA_TRY(alloc((size_t)m * 8, &w_.thetai));
  KA_TRY(alloc((size_t)m * 8, &w_.norms));
  KA_TRY(alloc(std::max({basis_work(m), sym_tri_work(m), nonsym_eig_work(m, std::min(nev_ + 1, m))}) * 8, &w_.ework));
  KA_TRY(alloc(tn_work_doubles(m, b, N) * 8, &w_.tnwork));
  KA_TRY(alloc(column_norms_work(N, std::max(ncol, b)) * 8, &w_.nwork));
  KA_TRY(alloc((size_t)b * 8, &w_.pnorm));
  {
    double* st = nullptr;
    KA_TRY(alloc(256, &st));
    w_.status = (int*)st;
  }
  th_.assign(m, 0.0);
  thi_.assign(m, 0.0);
  rn_.assign(m, 0.0);
  th_prev_.clear();
  thi_prev_.clear();
  pairs0_ = P_->pairs_total;
  HIP_TRY(fill_normal(w_.P, N, b, N, P_->d.seed, rng_counter_, s_));
  pw_ = (int)std::min<int64_t>(b, m);
  KA_TRY(orth_block(0, pw_));
  k_ = 0;
  return KA_OK;
}

int EigRun::pre_apply() {
  const int64_t N = P_->N;
  HIP_TRY(copy_cols(w_.P, N, w_.X + (size_t)k_ * N, N, N, pw_, s_));
  return apply_pre(P_, KA_APRIME, w_.X + (size_t)k_ * N, N, pw_, s_);
}

int EigRun::rayleigh_ritz(bool& stop) {
  const int64_t N = P_->N;
  const int m = m_max_;
  const int k = k_;
  int nk;
  int ns_status = 0;
  if (sym_) {
    nk = std::min(nev_, k);
    HIP_TRY(sym_eig_tri(w_.H, k, m, nk, w_.theta, w_.S, m, w_.ework, s_));
  } else {
    nk = std::min(nev_ + 1, k);
    HIP_TRY(nonsym_eig(w_.H, k, m, nk, w_.theta, w_.thetai, w_.S, m, w_.ework, w_.status, s_));
  }
  HIP_TRY(dgemm_nn(N, nk, k, 1.0, w_.X, N, w_.S, m, 0.0, w_.XS, N, s_));
  HIP_TRY(dgemm_nn(N, nk, k, 1.0, w_.AX, N, w_.S, m, 0.0, w_.AXS, N, s_));
  HIP_TRY(residual_combine(w_.AXS, w_.XS, N, nk, N, w_.theta, sym_ ? nullptr : w_.thetai, w_.R, s_));
  HIP_TRY(column_norms(w_.R, N, nk, N, w_.norms, w_.nwork, s_));
  HIP_TRY(hipMemcpyAsync(th_.data(), w_.theta, sizeof(double) * (sym_ ? k : nk), hipMemcpyDeviceToHost, s_));
  HIP_TRY(hipMemcpyAsync(rn_.data(), w_.norms, sizeof(double) * nk, hipMemcpyDeviceToHost, s_));
  if (!sym_) {
    HIP_TRY(hipMemcpyAsync(thi_.data(), w_.thetai, sizeof(double) * nk, hipMemcpyDeviceToHost, s_));
    HIP_TRY(hipMemcpyAsync(&ns_status, w_.status, sizeof(int), hipMemcpyDeviceToHost, s_));
  }
  HIP_TRY(hipStreamSynchronize(s_));
  ++cycles_;
  if (!sym_ && ns_status != 0) return fail(KA_ERR_SINGULAR, "Rayleigh-Ritz QR iteration did not converge");
  if (!sym_) {
    // a complex pair shares one residual (re and im parts of one unit vector)
    for (int i = 0; i + 1 < nk; ++i)
      if (thi_[i] > 0.0) {
        rn_[i] = rn_[i + 1] = std::sqrt(rn_[i] * rn_[i] + rn_[i + 1] * rn_[i + 1]);
        ++i;
      }
  }
  const double tau = 1e-2;
  // extend M to the end of its cluster (relative gap below 1e-6) or pair
  const int nlim = sym_ ? nk : std::min(nev_, k);
  Meff_ = std::min(M_, nlim);
  while (Meff_ < nlim && std::fabs(th_[Meff_ - 1] - th_[Meff_]) <= 1e-6 * std::fabs(th_[Meff_ - 1])) ++Meff_;
  if (!sym_ && Meff_ < nk && thi_[Meff_ - 1] > 0.0) ++Meff_;
  const double floor_ = std::max(tol_ * tau, noise_) * modulus(0);
  nconv_ = 0;
  floor_ok_ = 0;
  max_res_ = 0.0;
  max_imag_ = 0.0;
  for (int i = 0; i < Meff_; ++i) {
    const double crit = std::max(tol_ * modulus(i), floor_);
    const double rel = rn_[i] / std::max(modulus(i), tau * modulus(0));
    if (i < M_) {
      max_res_ = std::max(max_res_, rel);
      if (!sym_) max_imag_ = std::max(max_imag_, std::fabs(thi_[i]) / modulus(i));
    }
    bool ok = rn_[i] <= crit;
    // Ritz values below the noise floor cannot be resolved by the operator's
    // arithmetic: they are accepted by the floor alone (absolute error <= nu |theta_1|)
    if (sym_ && ok && rn_[i] > tol_ * modulus(i) && modulus(i) > noise_ * modulus(0)) {
      // accepted through the noise floor only: also require the Ritz value to be
      // accurate, |theta - lambda| <= r^2 / gap, to a tenth of tol on the floored
      // scale.  gap: distance to the nearest Ritz value (among all k) outside the
      // cluster of values that neither r nor the arithmetic noise can separate
      // from theta_i.
      const double sep = std::max({1e-6 * std::fabs(th_[i]), rn_[i], noise_ * modulus(0)});
      double gap = 1e300;
      for (int j = 0; j < k; ++j)
        if (std::fabs(th_[j] - th_[i]) > sep) gap = std::min(gap, std::fabs(th_[j] - th_[i]));
      ok = rn_[i] * rn_[i] <= 0.1 * tol_ * std::max(modulus(i), tau * modulus(0)) * gap;
    }
    // Non-symmetric A' (collocation): the eigenvalue error is first order in
    // r, so the floor alone certifies only |theta - lambda| ~ nu |theta_1|.
    // A pair accepted through it must also have kept its Ritz value, within a
    // tenth of the target, since the previous Rayleigh-Ritz step (so never in
    // the first cycle): the operator's arithmetic cannot resolve it further.
    if (!sym_ && ok && rn_[i] > tol_ * std::max(modulus(i), tau * modulus(0))) {
      ok = i < (int)th_prev_.size() &&
           std::hypot(th_[i] - th_prev_[i], thi_[i] - thi_prev_[i]) <=
               0.1 * tol_ * std::max(modulus(i), tau * modulus(0));
    }
    if (ok && nconv_ == i) {
      ++nconv_;
      // accepted although above tol on the floored scale: through the noise floor
      if (i < M_ && rel > tol_) ++floor_ok_;
    }
  }
  nret_ = sym_ ? nk : std::min(nk, Meff_ + 1);
  converged_ = nconv_ >= Meff_;
  if (!sym_) {
    th_prev_.assign(th_.begin(), th_.begin() + nk);
    thi_prev_.assign(thi_.begin(), thi_.begin() + nk);
  }
  // stagnation: three restart cycles without a 10% drop of the largest
  // scaled residual end the iteration (KA_NOT_CONVERGED, results valid)
  if (max_res_ < 0.9 * best_res_) {
    best_res_ = max_res_;
    stall_ = 0;
  } else {
    ++stall_;
  }
  if (verbose_) {
    double rmax = 0.0;
    for (int i = 0; i < Meff_; ++i) rmax = std::max(rmax, rn_[i] / modulus(0));
    std::fprintf(stderr, "[ka_eigs] cycle %d k %d matvecs %d nconv %d/%d max_rel %.3e max_abs/theta1 %.3e theta1 %.6e\n",
                 cycles_, k, matvecs_, nconv_, Meff_, max_res_, rmax, th_[0]);
  }
  if (converged_ || cycles_ >= maxit_ || full_ || stall_ >= 3) {
    stop = true;
    return KA_OK;
  }
  stop = false;
  // thick restart onto the leading Ritz vectors
  if (sym_) {
    HIP_TRY(copy_cols(w_.XS, N, w_.X, N, N, nk, s_));
    HIP_TRY(copy_cols(w_.AXS, N, w_.AX, N, N, nk, s_));
    hipLaunchKernelGGL(set_diag_kernel, dim3((nk * nk + 255) / 256), dim3(256), 0, s_, w_.H, m, nk, w_.theta);
    HIP_TRY(hipGetLastError());
    k_ = nk;
  } else {
    int nkeep = std::min(nev_, k);
    if (nkeep < nk && thi_[nkeep - 1] > 0.0) ++nkeep;
    // orthonormal basis of the kept Ritz vectors: W with S W orthonormal, by
    // pivoted Cholesky of G = S^T S (vectors dependent on the chosen ones to
    // kBasisCut are dropped), then once more on W1^T G W1, which restores the
    // orthonormality that the first pass loses to the conditioning of S
    HIP_TRY(dgemm_tn(nkeep, nkeep, k, 1.0, w_.S, m, w_.S, m, 0.0, w_.Gm, m, w_.tnwork, s_));
    HIP_TRY(orthonormal_basis(w_.Gm, nkeep, m, kBasisCut, w_.Wm, m, w_.ework, w_.status + 1, s_));
    int r1 = 0, good = 0;
    HIP_TRY(hipMemcpyAsync(&r1, w_.status + 1, sizeof(int), hipMemcpyDeviceToHost, s_));
    HIP_TRY(hipStreamSynchronize(s_));
    if (r1 < 1) return fail(KA_ERR_SINGULAR, "restart: the kept Ritz vectors span nothing");
    HIP_TRY(dgemm_nn(nkeep, r1, nkeep, 1.0, w_.Gm, m, w_.Wm, m, 0.0, w_.Hc, m, s_));                 // G W1
    HIP_TRY(dgemm_tn(r1, r1, nkeep, 1.0, w_.Wm, m, w_.Hc, m, 0.0, w_.Gm, m, w_.tnwork, s_));        // W1^T G W1
    HIP_TRY(orthonormal_basis(w_.Gm, r1, m, kBasisCut, w_.Hc, m, w_.ework, w_.status + 1, s_));     // W2
    HIP_TRY(hipMemcpyAsync(&good, w_.status + 1, sizeof(int), hipMemcpyDeviceToHost, s_));
    HIP_TRY(hipStreamSynchronize(s_));
    if (good < 1) return fail(KA_ERR_SINGULAR, "restart: the kept Ritz vectors span nothing");
    HIP_TRY(dgemm_nn(nkeep, good, r1, 1.0, w_.Wm, m, w_.Hc, m, 0.0, w_.Gm, m, s_));                  // W = W1 W2
    HIP_TRY(copy_cols(w_.Gm, m, w_.Wm, m, nkeep, good, s_));
    // X <- XS W, AX <- AXS W
    HIP_TRY(dgemm_nn(N, good, nkeep, 1.0, w_.XS, N, w_.Wm, m, 0.0, w_.T, N, s_));
    HIP_TRY(copy_cols(w_.T, N, w_.X, N, N, good, s_));
    HIP_TRY(dgemm_nn(N, good, nkeep, 1.0, w_.AXS, N, w_.Wm, m, 0.0, w_.T, N, s_));
    HIP_TRY(copy_cols(w_.T, N, w_.AX, N, N, good, s_));
    // H <- W^T S^T H S W
    HIP_TRY(dgemm_nn(k, nkeep, k, 1.0, w_.H, m, w_.S, m, 0.0, w_.Hc, m, s_));
    HIP_TRY(dgemm_tn(nkeep, nkeep, k, 1.0, w_.S, m, w_.Hc, m, 0.0, w_.Gm, m, w_.tnwork, s_));
    HIP_TRY(dgemm_nn(nkeep, good, nkeep, 1.0, w_.Gm, m, w_.Wm, m, 0.0, w_.Hc, m, s_));
    HIP_TRY(dgemm_tn(good, good, nkeep, 1.0, w_.Wm, m, w_.Hc, m, 0.0, w_.H, m, w_.tnwork, s_));
    k_ = good;
  }
  pw_ = P_->b;
  return KA_OK;
}

int EigRun::post_apply(bool& done) {
  const int64_t N = P_->N;
  const int b = P_->b;
  const int m = m_max_;
  done = false;
  KA_TRY(apply_post(P_, KA_APRIME, w_.AX + (size_t)k_ * N, N, pw_, s_));
  ++matvecs_;
  // H[0:k+pw, k:k+pw] = X^T AP
  HIP_TRY(dgemm_tn(k_ + pw_, pw_, N, 1.0, w_.X, N, w_.AX + (size_t)k_ * N, N, 0.0, w_.H + (size_t)k_ * m, m,
                   w_.tnwork, s_));
  if (sym_) {
    hipLaunchKernelGGL(symmetrize_block_kernel, dim3((pw_ * pw_ + 255) / 256), dim3(256), 0, s_, w_.H, m, k_, pw_);
    if (k_ > 0)
      hipLaunchKernelGGL(mirror_kernel, dim3((k_ * pw_ + 255) / 256), dim3(256), 0, s_, w_.H, m, k_, pw_);
    HIP_TRY(hipGetLastError());
  } else if (k_ > 0) {
    // new rows: H[k:k+pw, 0:k] = P^T A' X
    HIP_TRY(dgemm_tn(pw_, k_, N, 1.0, w_.X + (size_t)k_ * N, N, w_.AX, N, 0.0, w_.H + k_, m, w_.tnwork, s_));
  }
  k_ += pw_;
  // next pending block
  const int room = m - k_;
  const bool need_rr = full_ ? (k_ >= m) : (room < b);
  const int next_pw = full_ ? std::min(b, m - k_) : b;
  if (next_pw > 0) {
    HIP_TRY(copy_cols(w_.AX + (size_t)(k_ - pw_) * N, N, w_.P, N, N, std::min(pw_, next_pw), s_));
    if (next_pw > pw_)
      HIP_TRY(fill_normal(w_.P + (size_t)pw_ * N, N, next_pw - pw_, N, P_->d.seed, ++rng_counter_, s_));
    KA_TRY(orth_block(k_, next_pw));
  }
  if (!need_rr) {
    pw_ = next_pw;
    return KA_OK;
  }
  return rayleigh_ritz(done);
}

int EigRun::finish(double* lambda_host, double* V_dev, ka_info* info) {
  const int64_t N = P_->N;
  const int b = P_->b;
  if (full_) {
    converged_ = true;
    nconv_ = std::max(nconv_, Meff_);
  }
  // Galerkin: v = L^-T y (Z-orthonormal).  Collocation: v = y (unit 2-norm;
  // a genuine complex pair as re, im columns).  Imaginary parts at the
  // arithmetic noise level (a cluster split into a complex pair by rounding)
  // are reported as zero and both columns as real vectors.
  const int Mo = std::min(M_, nret_);
  std::vector<double> wi_out(std::max(Mo, 1), 0.0);
  if (!sym_) {
    const double real_tol = 10.0 * noise_;
    for (int i = 0; i < Mo; ++i) {
      const bool pair_start = thi_[i] > 0.0 && i + 1 < nret_;
      if (pair_start && std::fabs(thi_[i]) > real_tol * modulus(i)) {
        wi_out[i] = thi_[i];
        if (i + 1 < Mo) wi_out[i + 1] = thi_[i + 1];
        ++i;
      } else if (pair_start) {
        ++i;
      }
    }
  }
  for (int i = 0; i < Mo; ++i) {
    if (sym_) {
      lambda_host[i] = th_[i];
    } else {
      lambda_host[2 * i] = th_[i];
      lambda_host[2 * i + 1] = wi_out[i];
    }
  }
  for (int i = Mo; i < M_; ++i) {
    if (sym_) lambda_host[i] = 0.0;
    else lambda_host[2 * i] = lambda_host[2 * i + 1] = 0.0;
  }
  if (V_dev && Mo > 0) {
    if (sym_) {
      for (int c0 = 0; c0 < Mo; c0 += b) {
        const int nv = std::min(b, Mo - c0);
        KA_TRY(solve_block(P_, KA_LTINV, w_.XS + (size_t)c0 * N, N, nv, s_));
      }
      HIP_TRY(sign_fix(w_.XS, N, Mo, N, nullptr, s_));
    } else {
      // columns reported as real get unit norm each
      std::vector<double> nrm(Mo), sc(Mo);
      HIP_TRY(column_norms(w_.XS, N, Mo, N, w_.norms, w_.nwork, s_));
      HIP_TRY(hipMemcpyAsync(nrm.data(), w_.norms, sizeof(double) * Mo, hipMemcpyDeviceToHost, s_));
      HIP_TRY(hipStreamSynchronize(s_));
      for (int i = 0; i < Mo; ++i) sc[i] = (wi_out[i] == 0.0 && nrm[i] > 0.0) ? 1.0 / nrm[i] : 1.0;
      HIP_TRY(hipMemcpyAsync(w_.norms, sc.data(), sizeof(double) * Mo, hipMemcpyHostToDevice, s_));
      HIP_TRY(scale_cols(w_.XS, N, Mo, N, w_.norms, s_));
      HIP_TRY(hipMemcpyAsync(w_.thetai, wi_out.data(), sizeof(double) * Mo, hipMemcpyHostToDevice, s_));
      HIP_TRY(sign_fix(w_.XS, N, Mo, N, w_.thetai, s_));
    }
    HIP_TRY(copy_cols(w_.XS, N, V_dev, N, N, Mo, s_));
  }
  HIP_TRY(hipStreamSynchronize(s_));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start_).count();
  if (info) {
    info->iterations = cycles_;
    info->matvecs = matvecs_;
    info->converged = std::min(nconv_, M_);
    info->nev_computed = Meff_;
    info->max_residual = max_res_;
    info->max_imag_rel = max_imag_;
    info->seconds = secs;
    info->gamma_seconds = 0.0;
    info->pairs = P_->pairs_total - pairs0_;
    info->lambda_doubles = (int)lambda_doubles(P_->d, M_);
    info->floor_accepted = floor_ok_;
  }
  return converged_ ? KA_OK : KA_NOT_CONVERGED;
}

int eigs(Problem* P, int M, double tol, int maxit, double* lambda_host, double* V_dev, ka_info* info) {
  EigRun run(P, M, tol, maxit);
  KA_TRY(run.start());
  bool done = false;
  while (!done) {
    KA_TRY(run.pre_apply());
    KA_TRY(gamma_step(P, P->w32b, P->w32a, P->stream));
    KA_TRY(run.post_apply(done));
  }
  return run.finish(lambda_host, V_dev, info);
}

}  // namespace ka
