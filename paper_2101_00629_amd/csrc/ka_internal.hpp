// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ka.h"
#include "host_setup.hpp"

namespace ka {

// ---- kernel product -----------------------------------------------------
struct GammaLaunch {
  const float* xr;        // row points, stride xr_stride floats (x, y, z first)
  int xr_stride;
  const float* rs;        // optional row scale (nr)
  int64_t nr;
  const float* xc;        // column points
  int xc_stride;
  int64_t nc;
  const float* Y;         // nc x b, b contiguous
  float* Z;               // nr x b, b contiguous
  float* partial;         // split-K scratch, nsplit * nr * b floats
  uint4* ys;              // BF16X3: Y split into hi/lo BF16 MFMA fragments (gamma_split_y); filled by launch_gamma
  float coord_scale;      // applied to every coordinate on load
  float out_scale;        // sigma^2
  int nsplit;             // filled by launch_gamma
  int64_t cols_per_split; // filled by launch_gamma
  int64_t row_blocks;     // filled by launch_gamma
  int xcd_splits;         // filled by launch_gamma: > 0 selects the XCD-grouped 1-D grid
};

struct GammaPlan {
  int rows_per_block;
  int64_t row_blocks;
  int nsplit;
  int64_t cols_per_split;
  size_t partial_bytes;
  size_t ysplit_bytes;    // BF16X3: pre-split Y, ceil(nc / 64) * 64 * b * 4 bytes; 0 for FP32
  size_t work_bytes;      // scratch of one product: partials (256-byte aligned), then the pre-split Y
  int xcd_splits;         // 0, or the split count rounded up to the XCD count (grouped grid)
};

GammaPlan gamma_plan(int64_t nr, int64_t nc, int b, int precision);
// Start of the pre-split Y inside a product's scratch `work` (BF16X3), or nullptr.
uint4* gamma_ysplit_ptr(float* work, const GammaPlan& p);

// One kernel product of a batched launch, and one work item of it.
struct GammaJob {
  GammaLaunch a;    // nsplit / cols_per_split filled from gamma_plan
  int kernel;
};
struct GammaItem {
  int job;
  int rblk;
  int split;
};
int gamma_rows_per_block(int b);
hipError_t launch_gamma_batch(const GammaJob* jobs_dev, const GammaItem* items_dev, int n_items, int b,
                              int precision, hipStream_t s);
hipError_t launch_gamma_reduce(const float* partial, int nsplit, int64_t n, float* Z, hipStream_t s);
// BF16X3 pre-pass of a batched launch: splits Y of jobs [0, n_jobs) into their ys arrays.
hipError_t launch_gamma_split_jobs(const GammaJob* jobs_dev, int n_jobs, int b, hipStream_t s);
hipError_t launch_gamma(GammaLaunch a, int kernel, int b, int precision, hipStream_t s);
float kernel_coord_scale(int kernel, double ell);

// ---- Kronecker mode products -------------------------------------------
// A tensor with dims (n1, n2, n3) per vector and nv vectors.  Layout
// LAYOUT_COL: element (i, j) at i + j * ld (column-major block, the FP64 API
// layout); LAYOUT_PT: element (i, j) at i * ld + j (point-major, the kernel
// product's layout, ld = block size).  i = i1 + n1 (i2 + n2 i3).
enum { LAYOUT_COL = 0, LAYOUT_PT = 1 };

struct ModeArgs {
  const void* in;
  int in_layout;
  int64_t in_ld;          // column stride (COL) or point stride (PT)
  void* out;
  int out_layout;
  int64_t out_ld;
  int n_in[3];            // input dims
  int mode;               // 0, 1, 2
  int m;                  // output size along `mode`
  const void* mat;        // m x n_in[mode], row-major
  const void* matT;       // its transpose, n_in[mode] x m row-major (point-major layouts need it)
  int nv;                 // vectors
  const float* out_scale; // optional per-point scale of the output (output dims)
};

// TIn/TOut in {float, double}; the matrix and accumulation are TAcc.
hipError_t launch_mode_f64(const ModeArgs& a, hipStream_t s);                  // in/out/mat double
hipError_t launch_mode_f64_to_f32(const ModeArgs& a, hipStream_t s);           // in double, mat/out float
hipError_t launch_mode_f32(const ModeArgs& a, hipStream_t s);                  // all float
hipError_t launch_mode_f32_to_f64(const ModeArgs& a, hipStream_t s);           // in/mat float, out double
hipError_t launch_mode_f32in_f64(const ModeArgs& a, hipStream_t s);            // in float, mat/out double
// point-major FP32 (point stride ld_in) -> column-major FP64, divided by div[i] if div is not NULL
hipError_t cast_pt32_to_col64(const float* in, int64_t ld_in, double* out, int64_t ld_out, int64_t npts, int nv,
                              const double* div, hipStream_t s);
// FP64 layout changes: point-major (point stride ld) <-> column-major (column stride ld)
hipError_t pt64_to_col64(const double* in, int64_t ld_in, double* out, int64_t ld_out, int64_t npts, int nv,
                         hipStream_t s);
hipError_t col64_to_pt64(const double* in, int64_t ld_in, double* out, int64_t ld_out, int64_t npts, int nv,
                         hipStream_t s);

// ---- FP64 dense helpers (eigensolver) ----------------------------------
// C(m x n) = alpha * A^T B + beta * C, A: K x m (lda), B: K x n (ldb); split-K
// partials in `work` (>= dgemm_tn_work(m, n, K) doubles), fixed reduction order.
size_t dgemm_tn_work(int m, int n, int64_t K);
hipError_t dgemm_tn(int m, int n, int64_t K, double alpha, const double* A, int64_t lda,
                    const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                    double* work, hipStream_t s);
// C(M x n) = alpha * A B + beta * C, A: M x k (lda), B: k x n (ldb).
hipError_t dgemm_nn(int64_t M, int n, int k, double alpha, const double* A, int64_t lda,
                    const double* B, int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s);
// Small dense kernels, one workgroup each.
// ref (optional, n norms): a pivot below (kOrthKeep ref_j)^2 also counts as lost.
constexpr double kOrthKeep = 1e-9;
hipError_t chol_upper_inv(const double* G, int n, int ldg, double* Rinv, int ldr, int* status,
                          hipStream_t s, const double* ref = nullptr);
// Orthonormal basis of the span of vectors S from G = S^T S (n x n): W (n x
// rank, leading dimension ldw) with S W orthonormal, by diagonal-pivoted
// Cholesky stopped at the first pivot at or below cut * max G(i, i); rank to a
// device int.  work: basis_work(n) doubles.  The collocation thick restart.
hipError_t orthonormal_basis(const double* G, int n, int ldg, double cut, double* W, int ldw, double* work,
                             int* rank, hipStream_t s);
size_t basis_work(int n);
// Tridiagonal route (Householder, multisection, inverse iteration): the Galerkin
// Rayleigh-Ritz step.
// All n eigenvalues (theta, descending) and the eigenvectors of the nvec largest
// (S columns 0 .. nvec-1).
hipError_t sym_eig_tri(const double* H, int n, int ldh, int nvec, double* theta, double* S, int lds, double* work,
                       hipStream_t s);
size_t sym_tri_work(int n);
// All n eigenvalues (wr, wi; descending real part, a pair as consecutive entries
// with the positive imaginary part first) and the eigenvectors of the nvec
// leading ones (S columns; a pair as real and imaginary parts, extended by one
// column when a pair straddles nvec).  status: 0, or 1 if the QR iteration
// did not converge.
hipError_t nonsym_eig(const double* H, int n, int ldh, int nvec, double* wr, double* wi, double* S, int lds,
                      double* work, int* status, hipStream_t s);
size_t nonsym_eig_work(int n, int nvec_max);
hipError_t column_norms(const double* X, int64_t N, int n, int64_t ldx, double* out, double* work,
                        hipStream_t s);
size_t column_norms_work(int64_t N, int n);
hipError_t fill_normal(double* X, int64_t N, int n, int64_t ldx, uint64_t seed, uint64_t counter,
                       hipStream_t s);
hipError_t copy_cols(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t N, int n,
                     hipStream_t s);
hipError_t residual_combine(const double* AXS, const double* XS, int64_t N, int n, int64_t ld,
                            const double* wr, const double* wi, double* R, hipStream_t s);
hipError_t sign_fix(double* V, int64_t N, int n, int64_t ld, const double* wi, hipStream_t s);
hipError_t scale_cols(double* V, int64_t N, int n, int64_t ld, const double* scale, hipStream_t s);
// V[i + j ld] *= scale[i], i < N, j < n
hipError_t scale_rows(double* V, int64_t N, int n, int64_t ld, const double* scale, hipStream_t s);
hipError_t fill_zero_f32(float* p, int64_t n, hipStream_t s);

// ---- problem ----------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// A range of a server's device arena that one request's problem and solve
// allocate from, front to back; the server takes the range back whole.
struct Region {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
};

struct Problem {
  ka_desc d;
  Geometry geo;              // host copy of the domain map
  hipStream_t stream = nullptr;
  int device = 0;
  int N = 0, n[3] = {0, 0, 0};
  Vec tsol[3];                       // knot vectors of the solution space (host)
  int Nt = 0, nt[3] = {0, 0, 0};     // Galerkin interpolation space
  int64_t Nq = 0; int nq[3] = {0, 0, 0};  // collocation quadrature points
  int b = 16;
  float coord_scale = 1.f;
  float out_scale = 1.f;
  // device factors
  double* LinvT[3] = {nullptr, nullptr, nullptr};   // (L_k^-T) n x n  (Galerkin)
  double* Linv[3] = {nullptr, nullptr, nullptr};    // (L_k^-1)
  double* Zinv[3] = {nullptr, nullptr, nullptr};    // (Z_k^-1) (collocation LU inverse / Galerkin mass inverse)
  double* ZinvT[3] = {nullptr, nullptr, nullptr};   // (Z_k^-1)^T (the same array as Zinv where Z_k is symmetric)
  double* Zk[3] = {nullptr, nullptr, nullptr};      // Galerkin: mass matrices Z_k (n x n)
  float* T[3] = {nullptr, nullptr, nullptr};        // Galerkin: B~_k^-T M_k (nt x n); collocation: R_q,k (nq x n)
  float* TT[3] = {nullptr, nullptr, nullptr};       // transposes (n x nt)
  float* rows = nullptr;     // row points (x, y, z, 0), prescaled
  float* cols = nullptr;     // column points (Galerkin: == rows)
  float* rscale = nullptr;   // row scale (Galerkin: J; collocation on a NURBS volume: W at the collocation points)
  double* wrow64 = nullptr;  // collocation on a NURBS volume: W at the collocation points, FP64
  float* cscale = nullptr;   // column scale folded into Y (Galerkin: J, collocation: |det DF| W)
  int64_t n_rows = 0, n_cols = 0;
  // workspace
  double* w64a = nullptr;    // N x b FP64
  double* w64b = nullptr;
  float* w32a = nullptr;     // max(Nt, Nq, N) x b FP32
  float* w32b = nullptr;
  float* gpart = nullptr;    // split-K partials
  size_t gpart_bytes = 0;
  Region region;             // base set: every allocation comes from this range (served requests)
  std::vector<DevBuf> allocs; // hipMalloc'd buffers owned by the problem (freed with it)
  size_t device_bytes = 0;
  // profiling
  bool profile = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  int prof_launches = 0;
  double prof_ms = 0.0;
  double prof_pairs = 0.0;
  double pairs_total = 0.0;
  // eigensolver workspace: allocated by the first ka_eigs, kept between
  // calls, replaced by a larger one only when a call needs more
  void* eig_buf = nullptr;
  size_t eig_buf_bytes = 0;
  // K-L sampling: a workspace kept between calls (grown on demand, freed
  // with the problem), and the collocation norm data that depend on the
  // problem only: quadrature weights times |det DF| / W^2 at the Gauss
  // points and the trial factors there (kept in allocs)
  void* kl_buf = nullptr;
  size_t kl_bytes = 0;
  double* kl_omega = nullptr;
  double* kl_Eq[3] = {nullptr, nullptr, nullptr};
  int kl_mq[3] = {0, 0, 0};
};

void set_error(const std::string& msg);
const char* last_error_cstr();
int fail(int code, const std::string& msg);

// device-side operator pieces (api.cpp)
int apply_block(Problem* P, int form, const double* X, int64_t ldx, double* Y, int64_t ldy, int nv,
                hipStream_t s);
int solve_block(Problem* P, int op, double* X, int64_t ld, int nv, hipStream_t s);
int apply_pre(Problem* P, int form, const double* X, int64_t ldx, int nv, hipStream_t s);
int apply_post(Problem* P, int form, double* Y, int64_t ldy, int nv, hipStream_t s);
GammaLaunch gamma_job(Problem* P);
int gamma_step(Problem* P, const float* Y, float* Z, hipStream_t s);
// Device memory for a problem: from its region when it has one, else
// hipMalloc (recorded in allocs).  nullptr when it does not fit or fails.
void* problem_alloc(Problem* P, size_t bytes);
// region: optional range every allocation of the problem comes from.
int setup_problem(const ka_desc* d, hipStream_t stream, Problem** out, const Region* region = nullptr);
int footprint(const ka_desc* d, size_t* bytes);
// N, Ntilde, Nquad that setup_problem would produce (host only).
int desc_sizes(const ka_desc* d, int64_t* N, int64_t* Nt, int64_t* Nq);
void destroy_problem(Problem* P);
int eigs(Problem* P, int M, double tol, int maxit, double* lambda_host, double* V_dev, ka_info* info);
// Doubles ka_eigs writes to lambda_host for M eigenvalues: M, or 2M (re, im) for collocation.
int64_t lambda_doubles(const ka_desc& d, int M);

}  // namespace ka
