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
//   leading nev Ritz vectors (X <- X S, AX <- AX S, H <- diag(theta)).
// Galerkin (symmetric A'): parallel Jacobi on H.  Collocation (A' = Z^-1 A,
// non-symmetric): Hessenberg QR on H, restart onto an orthonormal basis of
// the wanted Ritz vectors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "ka_internal.hpp"

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

struct EigWork {
  double *X = nullptr, *AX = nullptr, *P = nullptr, *XS = nullptr, *AXS = nullptr, *R = nullptr, *T = nullptr;
  double *H = nullptr, *Hc = nullptr, *C = nullptr, *G = nullptr, *Rinv = nullptr, *theta = nullptr,
         *thetai = nullptr, *S = nullptr, *norms = nullptr, *ework = nullptr, *tnwork = nullptr,
         *nwork = nullptr;
  int* status = nullptr;
};

// small device kernels local to the solver
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

class Solver {
 public:
  Solver(Problem* P) : P_(P), s_(P->stream) {}
  ~Solver() {}
  int run(int M, double tol, int maxit, double* lambda_host, double* V_dev, ka_info* info);

 private:
  int alloc(size_t bytes, double** out);
  int orth_block(int k, int pw, uint64_t& rng_counter);
  Problem* P_;
  hipStream_t s_;
  EigWork w_;
  std::vector<DevBuf> bufs_;
};

int Solver::alloc(size_t bytes, double** out) {
  bytes = (bytes + 255) / 256 * 256;
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(KA_ERR_OOM, "eigensolver workspace allocation failed");
  P_->eig_allocs.push_back({p, bytes});
  P_->eig_bytes += bytes;
  *out = (double*)p;
  return KA_OK;
}

// Orthonormalise P (N x pw) against X[:, :k] (block CGS twice) and within
// itself (Cholesky-QR twice).  Rank-deficient blocks are redrawn at random.
int Solver::orth_block(int k, int pw, uint64_t& rng_counter) {
  const int64_t N = P_->N;
  for (int attempt = 0; attempt < 4; ++attempt) {
    if (k > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        HIP_TRY(dgemm_tn(k, pw, N, 1.0, w_.X, N, w_.P, N, 0.0, w_.C, k, w_.tnwork, s_));
        HIP_TRY(dgemm_nn(N, pw, k, -1.0, w_.X, N, w_.C, k, 1.0, w_.P, N, s_));
      }
    }
    int bad = 0;
    for (int pass = 0; pass < 2 && !bad; ++pass) {
      HIP_TRY(dgemm_tn(pw, pw, N, 1.0, w_.P, N, w_.P, N, 0.0, w_.G, pw, w_.tnwork, s_));
      HIP_TRY(chol_upper_inv(w_.G, pw, pw, w_.Rinv, pw, w_.status, s_));
      HIP_TRY(dgemm_nn(N, pw, pw, 1.0, w_.P, N, w_.Rinv, pw, 0.0, w_.T, N, s_));
      HIP_TRY(copy_cols(w_.T, N, w_.P, N, N, pw, s_));
      int st = 0;
      HIP_TRY(hipMemcpyAsync(&st, w_.status, sizeof(int), hipMemcpyDeviceToHost, s_));
      HIP_TRY(hipStreamSynchronize(s_));
      bad = st;
    }
    if (!bad) return KA_OK;
    // Krylov space exhausted along some direction: continue with random ones
    HIP_TRY(fill_normal(w_.P, N, pw, N, P_->d.seed, ++rng_counter, s_));
  }
  return fail(KA_ERR_SINGULAR, "could not extend the Krylov basis");
}

int Solver::run(int M, double tol, int maxit, double* lambda_host, double* V_dev, ka_info* info) {
  const auto t_start = std::chrono::steady_clock::now();
  const bool sym = P_->d.method == KA_GALERKIN_IBQ;
  const int64_t N = P_->N;
  const int b = P_->b;
  if (M < 1 || M > N) return fail(KA_ERR_ARG, "M must be in 1..N");
  if (!sym) return fail(KA_ERR_STATE, "collocation eigensolve is not available in this build");
  const double tau = 1e-2;
  if (!(tol > 0)) tol = 1e-6;
  if (maxit <= 0) maxit = 100;

  // basis sizes
  int nev = (int)std::min<int64_t>(N, (int64_t)M + b);
  const int nb = std::max(2, (nev + 2 * b - 1) / (2 * b));
  int m_max = nev + nb * b;
  bool full = false;
  if ((int64_t)m_max >= N) {   // small problem: the Krylov space becomes the whole space
    m_max = (int)N;
    full = true;
  }
  if (m_max > 1000) return fail(KA_ERR_ARG, "M too large for the dense Rayleigh-Ritz (M + block <= ~600)");

  // workspace
  KA_TRY(alloc((size_t)N * m_max * 8, &w_.X));
  KA_TRY(alloc((size_t)N * m_max * 8, &w_.AX));
  KA_TRY(alloc((size_t)N * b * 8, &w_.P));
  KA_TRY(alloc((size_t)N * std::max(nev, b) * 8, &w_.T));
  KA_TRY(alloc((size_t)N * nev * 8, &w_.XS));
  KA_TRY(alloc((size_t)N * nev * 8, &w_.AXS));
  KA_TRY(alloc((size_t)N * nev * 8, &w_.R));
  KA_TRY(alloc((size_t)m_max * m_max * 8, &w_.H));
  KA_TRY(alloc((size_t)m_max * b * 8, &w_.C));
  KA_TRY(alloc((size_t)b * b * 8, &w_.G));
  KA_TRY(alloc((size_t)b * b * 8, &w_.Rinv));
  KA_TRY(alloc((size_t)m_max * 8, &w_.theta));
  KA_TRY(alloc((size_t)m_max * 8, &w_.thetai));
  KA_TRY(alloc((size_t)m_max * m_max * 8, &w_.S));
  KA_TRY(alloc((size_t)m_max * 8, &w_.norms));
  KA_TRY(alloc(sym_eig_work(m_max) * 8, &w_.ework));
  size_t tnw = 0;
  for (int m = 1; m <= m_max; ++m) {
    tnw = std::max(tnw, dgemm_tn_work(m, b, N));
    tnw = std::max(tnw, dgemm_tn_work(b, m, N));
  }
  KA_TRY(alloc(tnw * 8, &w_.tnwork));
  KA_TRY(alloc(column_norms_work(N, nev) * 8, &w_.nwork));
  {
    double* st = nullptr;
    KA_TRY(alloc(256, &st));
    w_.status = (int*)st;
  }
  const double pairs0 = P_->pairs_total;

  uint64_t rng_counter = 0;
  HIP_TRY(fill_normal(w_.P, N, b, N, P_->d.seed, rng_counter, s_));
  int pw = (int)std::min<int64_t>(b, m_max);
  KA_TRY(orth_block(0, pw, rng_counter));

  int k = 0, cycles = 0, matvecs = 0, nconv = 0, Meff = M;
  double max_res = 0.0;
  std::vector<double> th(m_max), rn(m_max);
  int nret = 0;
  bool converged = false;
  while (true) {
    // append the pending block and apply A'
    HIP_TRY(copy_cols(w_.P, N, w_.X + (size_t)k * N, N, N, pw, s_));
    KA_TRY(apply_block(P_, KA_APRIME, w_.X + (size_t)k * N, N, w_.AX + (size_t)k * N, N, pw, s_));
    ++matvecs;
    // H[0:k+pw, k:k+pw] = X^T AP ; mirror into H[k:k+pw, 0:k]
    HIP_TRY(dgemm_tn(k + pw, pw, N, 1.0, w_.X, N, w_.AX + (size_t)k * N, N, 0.0, w_.H + (size_t)k * m_max, m_max,
                     w_.tnwork, s_));
    hipLaunchKernelGGL(symmetrize_block_kernel, dim3((pw * pw + 255) / 256), dim3(256), 0, s_, w_.H, m_max, k, pw);
    if (k > 0)
      hipLaunchKernelGGL(mirror_kernel, dim3((k * pw + 255) / 256), dim3(256), 0, s_, w_.H, m_max, k, pw);
    HIP_TRY(hipGetLastError());
    k += pw;
    // next pending block
    const int room = m_max - k;
    const bool need_rr = full ? (k >= m_max) : (room < b);
    int next_pw = full ? std::min(b, m_max - k) : b;
    if (next_pw > 0) {
      HIP_TRY(copy_cols(w_.AX + (size_t)(k - pw) * N, N, w_.P, N, N, std::min(pw, next_pw), s_));
      if (next_pw > pw) HIP_TRY(fill_normal(w_.P + (size_t)pw * N, N, next_pw - pw, N, P_->d.seed, ++rng_counter, s_));
      KA_TRY(orth_block(k, next_pw, rng_counter));
    }
    if (!need_rr) {
      pw = next_pw;
      continue;
    }
    // Rayleigh-Ritz
    HIP_TRY(sym_eig(w_.H, k, m_max, w_.theta, w_.S, m_max, w_.ework, s_));
    const int nk = std::min(nev, k);
    HIP_TRY(dgemm_nn(N, nk, k, 1.0, w_.X, N, w_.S, m_max, 0.0, w_.XS, N, s_));
    HIP_TRY(dgemm_nn(N, nk, k, 1.0, w_.AX, N, w_.S, m_max, 0.0, w_.AXS, N, s_));
    HIP_TRY(residual_combine(w_.AXS, w_.XS, N, nk, N, w_.theta, nullptr, w_.R, s_));
    HIP_TRY(column_norms(w_.R, N, nk, N, w_.norms, w_.nwork, s_));
    HIP_TRY(hipMemcpyAsync(th.data(), w_.theta, sizeof(double) * nk, hipMemcpyDeviceToHost, s_));
    HIP_TRY(hipMemcpyAsync(rn.data(), w_.norms, sizeof(double) * nk, hipMemcpyDeviceToHost, s_));
    HIP_TRY(hipStreamSynchronize(s_));
    ++cycles;
    // extend M to the end of its cluster (relative gap below 1e-6)
    Meff = std::min(M, nk);
    while (Meff < nk && std::fabs(th[Meff - 1] - th[Meff]) <= 1e-6 * std::fabs(th[Meff - 1])) ++Meff;
    const double floor_ = tau * std::fabs(th[0]);
    nconv = 0;
    max_res = 0.0;
    for (int i = 0; i < Meff; ++i) {
      const double rel = rn[i] / std::max(std::fabs(th[i]), floor_);
      if (i < M) max_res = std::max(max_res, rel);
      if (rel <= tol && nconv == i) ++nconv;
    }
    nret = nk;
    converged = nconv >= Meff;
    if (converged || cycles >= maxit || full) break;
    // thick restart
    HIP_TRY(copy_cols(w_.XS, N, w_.X, N, N, nk, s_));
    HIP_TRY(copy_cols(w_.AXS, N, w_.AX, N, N, nk, s_));
    hipLaunchKernelGGL(set_diag_kernel, dim3((nk * nk + 255) / 256), dim3(256), 0, s_, w_.H, m_max, nk, w_.theta);
    HIP_TRY(hipGetLastError());
    k = nk;
    pw = b;
  }
  if (full) converged = true, nconv = std::max(nconv, Meff);

  // outputs: eigenvalues, eigenvectors v = L^-T y (Z-orthonormal)
  const int Mo = std::min(M, nret);
  for (int i = 0; i < Mo; ++i) lambda_host[i] = th[i];
  for (int i = Mo; i < M; ++i) lambda_host[i] = 0.0;
  if (V_dev) {
    for (int c0 = 0; c0 < Mo; c0 += b) {
      const int nv = std::min(b, Mo - c0);
      KA_TRY(solve_block(P_, KA_LTINV, w_.XS + (size_t)c0 * N, N, nv, s_));
    }
    HIP_TRY(sign_fix(w_.XS, N, Mo, N, nullptr, s_));
    HIP_TRY(copy_cols(w_.XS, N, V_dev, N, N, Mo, s_));
  }
  HIP_TRY(hipStreamSynchronize(s_));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (info) {
    info->iterations = cycles;
    info->matvecs = matvecs;
    info->converged = std::min(nconv, M);
    info->nev_computed = Meff;
    info->max_residual = max_res;
    info->max_imag_rel = 0.0;
    info->seconds = secs;
    info->gamma_seconds = 0.0;
    info->pairs = P_->pairs_total - pairs0;
  }
  return converged ? KA_OK : KA_NOT_CONVERGED;
}

}  // namespace

int eigs(Problem* P, int M, double tol, int maxit, double* lambda_host, double* V_dev, ka_info* info) {
  int rc;
  {
    Solver S(P);
    rc = S.run(M, tol, maxit, lambda_host, V_dev, info);
  }
  // release the solver workspace
  (void)hipStreamSynchronize(P->stream);
  for (auto& b : P->eig_allocs) (void)hipFree(b.p);
  P->eig_allocs.clear();
  P->eig_bytes = 0;
  return rc;
}

}  // namespace ka
