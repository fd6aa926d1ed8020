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
#include <cstdio>
#include <cstdlib>
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
         *nwork = nullptr, *Wm = nullptr, *Gm = nullptr;
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

__global__ void inv_sqrt_kernel(const double* g, int n, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = g[i] > 0.0 ? 1.0 / sqrt(g[i]) : 0.0;
}

class Solver {
 public:
  Solver(Problem* P) : P_(P), s_(P->stream) {
    const char* v = std::getenv("KA_VERBOSE");
    verbose_ = v && v[0] && v[0] != '0';
  }
  ~Solver() {}
  int run(int M, double tol, int maxit, double* lambda_host, double* V_dev, ka_info* info);

 private:
  int alloc(size_t bytes, double** out);
  int orth_block(int k, int pw, uint64_t& rng_counter);
  Problem* P_;
  hipStream_t s_;
  EigWork w_;
  std::vector<DevBuf> bufs_;
  bool verbose_ = false;
  double noise_ = 0.0;
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
  const double tau = 1e-2;
  // Residuals of an operator applied in FP32 (or split BF16) cannot fall
  // below a few units of its rounding times |theta_1|; below that level the
  // Ritz values no longer move (symmetric case: error ~ r^2 / gap).
  noise_ = P_->d.precision == KA_FP32 ? 4e-6 : 1e-4;
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
  const int ncol = nev + 1;   // room for a complex pair that straddles nev
  KA_TRY(alloc((size_t)N * std::max(ncol, b) * 8, &w_.T));
  KA_TRY(alloc((size_t)N * ncol * 8, &w_.XS));
  KA_TRY(alloc((size_t)N * ncol * 8, &w_.AXS));
  KA_TRY(alloc((size_t)N * ncol * 8, &w_.R));
  KA_TRY(alloc((size_t)m_max * m_max * 8, &w_.Hc));
  KA_TRY(alloc((size_t)m_max * m_max * 8, &w_.Wm));
  KA_TRY(alloc((size_t)m_max * m_max * 8, &w_.Gm));
  KA_TRY(alloc((size_t)m_max * m_max * 8, &w_.H));
  KA_TRY(alloc((size_t)m_max * b * 8, &w_.C));
  KA_TRY(alloc((size_t)b * b * 8, &w_.G));
  KA_TRY(alloc((size_t)b * b * 8, &w_.Rinv));
  KA_TRY(alloc((size_t)m_max * 8, &w_.theta));
  KA_TRY(alloc((size_t)m_max * 8, &w_.thetai));
  KA_TRY(alloc((size_t)m_max * m_max * 8, &w_.S));
  KA_TRY(alloc((size_t)m_max * 8, &w_.norms));
  KA_TRY(alloc(std::max(sym_eig_work(m_max), nonsym_eig_work(m_max)) * 8, &w_.ework));
  size_t tnw = (size_t)m_max * m_max;
  for (int m = 1; m <= m_max; ++m) {
    tnw = std::max(tnw, dgemm_tn_work(m, b, N));
    tnw = std::max(tnw, dgemm_tn_work(b, m, N));
  }
  KA_TRY(alloc(tnw * 8, &w_.tnwork));
  KA_TRY(alloc(column_norms_work(N, ncol) * 8, &w_.nwork));
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

  int k = 0, cycles = 0, matvecs = 0, nconv = 0, Meff = M, ns_status = 0;
  double max_res = 0.0, max_imag = 0.0;
  std::vector<double> th(m_max), rn(m_max), thi(m_max, 0.0);
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
    if (sym) {
      hipLaunchKernelGGL(symmetrize_block_kernel, dim3((pw * pw + 255) / 256), dim3(256), 0, s_, w_.H, m_max, k, pw);
      if (k > 0)
        hipLaunchKernelGGL(mirror_kernel, dim3((k * pw + 255) / 256), dim3(256), 0, s_, w_.H, m_max, k, pw);
      HIP_TRY(hipGetLastError());
    } else if (k > 0) {
      // new rows: H[k:k+pw, 0:k] = P^T A' X
      HIP_TRY(dgemm_tn(pw, k, N, 1.0, w_.X + (size_t)k * N, N, w_.AX, N, 0.0, w_.H + k, m_max, w_.tnwork, s_));
    }
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
    int nk;
    if (sym) {
      HIP_TRY(sym_eig(w_.H, k, m_max, w_.theta, w_.S, m_max, w_.ework, s_));
      nk = std::min(nev, k);
    } else {
      HIP_TRY(nonsym_eig(w_.H, k, m_max, w_.theta, w_.thetai, w_.S, m_max, w_.ework, w_.status, s_));
      nk = std::min(nev + 1, k);
    }
    HIP_TRY(dgemm_nn(N, nk, k, 1.0, w_.X, N, w_.S, m_max, 0.0, w_.XS, N, s_));
    HIP_TRY(dgemm_nn(N, nk, k, 1.0, w_.AX, N, w_.S, m_max, 0.0, w_.AXS, N, s_));
    HIP_TRY(residual_combine(w_.AXS, w_.XS, N, nk, N, w_.theta, sym ? nullptr : w_.thetai, w_.R, s_));
    HIP_TRY(column_norms(w_.R, N, nk, N, w_.norms, w_.nwork, s_));
    HIP_TRY(hipMemcpyAsync(th.data(), w_.theta, sizeof(double) * nk, hipMemcpyDeviceToHost, s_));
    HIP_TRY(hipMemcpyAsync(rn.data(), w_.norms, sizeof(double) * nk, hipMemcpyDeviceToHost, s_));
    if (!sym) {
      HIP_TRY(hipMemcpyAsync(thi.data(), w_.thetai, sizeof(double) * nk, hipMemcpyDeviceToHost, s_));
      HIP_TRY(hipMemcpyAsync(&ns_status, w_.status, sizeof(int), hipMemcpyDeviceToHost, s_));
    }
    HIP_TRY(hipStreamSynchronize(s_));
    ++cycles;
    if (!sym && ns_status != 0) return fail(KA_ERR_SINGULAR, "Rayleigh-Ritz QR iteration did not converge");
    if (!sym) {
      // a complex pair shares one residual (re and im parts of one unit vector)
      for (int i = 0; i + 1 < nk; ++i)
        if (thi[i] > 0.0) {
          rn[i] = rn[i + 1] = std::sqrt(rn[i] * rn[i] + rn[i + 1] * rn[i + 1]);
          ++i;
        }
    }
    auto modulus = [&](int i) { return sym ? std::fabs(th[i]) : std::hypot(th[i], thi[i]); };
    // extend M to the end of its cluster (relative gap below 1e-6) or pair
    const int nlim = sym ? nk : std::min(nev, k);
    Meff = std::min(M, nlim);
    while (Meff < nlim && std::fabs(th[Meff - 1] - th[Meff]) <= 1e-6 * std::fabs(th[Meff - 1])) ++Meff;
    if (!sym && Meff < nk && thi[Meff - 1] > 0.0) ++Meff;
    const double floor_ = std::max(tol * tau, noise_) * modulus(0);
    nconv = 0;
    max_res = 0.0;
    max_imag = 0.0;
    for (int i = 0; i < Meff; ++i) {
      const double crit = std::max(tol * modulus(i), floor_);
      const double rel = rn[i] / std::max(modulus(i), tau * modulus(0));
      if (i < M) {
        max_res = std::max(max_res, rel);
        if (!sym) max_imag = std::max(max_imag, std::fabs(thi[i]) / modulus(i));
      }
      if (rn[i] <= crit && nconv == i) ++nconv;
    }
    nret = sym ? nk : std::min(nk, Meff + 1);
    converged = nconv >= Meff;
    if (verbose_) {
      double rmax = 0.0;
      for (int i = 0; i < Meff; ++i) rmax = std::max(rmax, rn[i] / modulus(0));
      std::fprintf(stderr, "[ka_eigs] cycle %d k %d matvecs %d nconv %d/%d max_rel %.3e max_abs/theta1 %.3e theta1 %.6e\n",
                   cycles, k, matvecs, nconv, Meff, max_res, rmax, th[0]);
    }
    if (converged || cycles >= maxit || full) break;
    // thick restart onto the leading Ritz vectors
    if (sym) {
      HIP_TRY(copy_cols(w_.XS, N, w_.X, N, N, nk, s_));
      HIP_TRY(copy_cols(w_.AXS, N, w_.AX, N, N, nk, s_));
      hipLaunchKernelGGL(set_diag_kernel, dim3((nk * nk + 255) / 256), dim3(256), 0, s_, w_.H, m_max, nk, w_.theta);
      HIP_TRY(hipGetLastError());
      k = nk;
    } else {
      int nkeep = std::min(nev, k);
      if (nkeep < nk && thi[nkeep - 1] > 0.0) ++nkeep;
      // orthonormal basis of the kept Ritz vectors: W = V Lambda^-1/2 from S^T S = V Lambda V^T
      HIP_TRY(dgemm_tn(nkeep, nkeep, k, 1.0, w_.S, m_max, w_.S, m_max, 0.0, w_.Gm, m_max, w_.tnwork, s_));
      HIP_TRY(sym_eig(w_.Gm, nkeep, m_max, w_.norms, w_.Wm, m_max, w_.ework, s_));
      std::vector<double> gl(nkeep);
      HIP_TRY(hipMemcpyAsync(gl.data(), w_.norms, sizeof(double) * nkeep, hipMemcpyDeviceToHost, s_));
      HIP_TRY(hipStreamSynchronize(s_));
      int good = 0;
      while (good < nkeep && gl[good] > 1e-12 * gl[0]) ++good;
      hipLaunchKernelGGL(inv_sqrt_kernel, dim3((good + 63) / 64), dim3(64), 0, s_, w_.norms, good, w_.norms);
      HIP_TRY(hipGetLastError());
      HIP_TRY(scale_cols(w_.Wm, nkeep, good, m_max, w_.norms, s_));
      // X <- XS W, AX <- AXS W
      HIP_TRY(dgemm_nn(N, good, nkeep, 1.0, w_.XS, N, w_.Wm, m_max, 0.0, w_.T, N, s_));
      HIP_TRY(copy_cols(w_.T, N, w_.X, N, N, good, s_));
      HIP_TRY(dgemm_nn(N, good, nkeep, 1.0, w_.AXS, N, w_.Wm, m_max, 0.0, w_.T, N, s_));
      HIP_TRY(copy_cols(w_.T, N, w_.AX, N, N, good, s_));
      // H <- W^T S^T H S W
      HIP_TRY(dgemm_nn(k, nkeep, k, 1.0, w_.H, m_max, w_.S, m_max, 0.0, w_.Hc, m_max, s_));
      HIP_TRY(dgemm_tn(nkeep, nkeep, k, 1.0, w_.S, m_max, w_.Hc, m_max, 0.0, w_.Gm, m_max, w_.tnwork, s_));
      HIP_TRY(dgemm_nn(nkeep, good, nkeep, 1.0, w_.Gm, m_max, w_.Wm, m_max, 0.0, w_.Hc, m_max, s_));
      HIP_TRY(dgemm_tn(good, good, nkeep, 1.0, w_.Wm, m_max, w_.Hc, m_max, 0.0, w_.H, m_max, w_.tnwork, s_));
      k = good;
    }
    pw = b;
  }
  if (full) converged = true, nconv = std::max(nconv, Meff);

  // outputs.  Galerkin: v = L^-T y (Z-orthonormal).  Collocation: v = y
  // (unit 2-norm; complex pairs as re, im columns).
  const int Mo = std::min(M, nret);
  for (int i = 0; i < Mo; ++i) {
    if (sym) {
      lambda_host[i] = th[i];
    } else {
      lambda_host[2 * i] = th[i];
      lambda_host[2 * i + 1] = thi[i];
    }
  }
  for (int i = Mo; i < M; ++i) {
    if (sym) lambda_host[i] = 0.0;
    else lambda_host[2 * i] = lambda_host[2 * i + 1] = 0.0;
  }
  if (V_dev && Mo > 0) {
    if (sym) {
      for (int c0 = 0; c0 < Mo; c0 += b) {
        const int nv = std::min(b, Mo - c0);
        KA_TRY(solve_block(P_, KA_LTINV, w_.XS + (size_t)c0 * N, N, nv, s_));
      }
    }
    HIP_TRY(sign_fix(w_.XS, N, Mo, N, sym ? nullptr : w_.thetai, s_));
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
    info->max_imag_rel = max_imag;
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
