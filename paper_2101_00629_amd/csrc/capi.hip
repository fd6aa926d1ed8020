// extern "C" surface of the library (declared in include/ka.h).
#include <hip/hip_runtime.h>

#include <string>

#include "ka_internal.hpp"

using namespace ka;

extern "C" {

const char* ka_last_error(void) { return last_error_cstr(); }

int ka_setup(const ka_desc* desc, void* stream, ka_problem** out) {
  if (!out) return fail(KA_ERR_ARG, "out is NULL");
  *out = nullptr;
  Problem* P = nullptr;
  const int rc = setup_problem(desc, (hipStream_t)stream, &P);
  if (rc == KA_OK) *out = reinterpret_cast<ka_problem*>(P);
  return rc;
}

int ka_size(const ka_problem* p, int64_t* N, int64_t* Ntilde, int64_t* Nquad, size_t* device_bytes) {
  const Problem* P = reinterpret_cast<const Problem*>(p);
  if (!P) return fail(KA_ERR_ARG, "problem is NULL");
  if (N) *N = P->N;
  if (Ntilde) *Ntilde = P->Nt;
  if (Nquad) *Nquad = P->Nq;
  if (device_bytes) *device_bytes = P->device_bytes + P->eig_buf_bytes + P->kl_bytes;
  return KA_OK;
}

int ka_desc_size(const ka_desc* desc, int64_t* N, int64_t* Ntilde, int64_t* Nquad) {
  return desc_sizes(desc, N, Ntilde, Nquad);
}

int ka_footprint(const ka_desc* desc, size_t* device_bytes) {
  if (!device_bytes) return fail(KA_ERR_ARG, "device_bytes is NULL");
  return footprint(desc, device_bytes);
}

int ka_apply_A(ka_problem* p, int form, const double* X_dev, int64_t ldx, double* Y_dev, int64_t ldy, int nvec,
               void* stream) {
  Problem* P = reinterpret_cast<Problem*>(p);
  if (!P) return fail(KA_ERR_ARG, "problem is NULL");
  if (form != KA_A && form != KA_APRIME) return fail(KA_ERR_ARG, "bad form");
  if (nvec < 0 || ldx < P->N || ldy < P->N) return fail(KA_ERR_ARG, "bad nvec or leading dimension");
  if (nvec > 0 && (!X_dev || !Y_dev)) return fail(KA_ERR_ARG, "NULL block");
  for (int c0 = 0; c0 < nvec; c0 += P->b) {
    const int nv = nvec - c0 < P->b ? nvec - c0 : P->b;
    const int rc = apply_block(P, form, X_dev + (size_t)c0 * ldx, ldx, Y_dev + (size_t)c0 * ldy, ldy, nv,
                               (hipStream_t)stream);
    if (rc) return rc;
  }
  return KA_OK;
}

int ka_solve_Z(ka_problem* p, int op, double* X_dev, int64_t ld, int nvec, void* stream) {
  Problem* P = reinterpret_cast<Problem*>(p);
  if (!P) return fail(KA_ERR_ARG, "problem is NULL");
  if (op != KA_ZINV && op != KA_LINV && op != KA_LTINV) return fail(KA_ERR_ARG, "bad op");
  if (nvec < 0 || ld < P->N) return fail(KA_ERR_ARG, "bad nvec or leading dimension");
  if (nvec > 0 && !X_dev) return fail(KA_ERR_ARG, "NULL block");
  for (int c0 = 0; c0 < nvec; c0 += P->b) {
    const int nv = nvec - c0 < P->b ? nvec - c0 : P->b;
    const int rc = solve_block(P, op, X_dev + (size_t)c0 * ld, ld, nv, (hipStream_t)stream);
    if (rc) return rc;
  }
  return KA_OK;
}

int ka_eigs(ka_problem* p, int M, double tol, int maxit, double* lambda_host, int64_t lambda_len, double* V_dev,
            ka_info* info) {
  Problem* P = reinterpret_cast<Problem*>(p);
  if (!P) return fail(KA_ERR_ARG, "problem is NULL");
  if (!lambda_host) return fail(KA_ERR_ARG, "lambda_host is NULL");
  if (M < 1 || M > P->N) return fail(KA_ERR_ARG, "M must be in 1..N");
  if (lambda_len < lambda_doubles(P->d, M))
    return fail(KA_ERR_ARG, "lambda_host holds " + std::to_string(lambda_len) + " doubles, the solve writes " +
                                std::to_string(lambda_doubles(P->d, M)));
  return eigs(P, M, tol, maxit, lambda_host, V_dev, info);
}

size_t ka_gamma_workspace(int64_t nr, int64_t nc, int b, int precision) {
  if (nr <= 0 || nc <= 0) return 0;
  return gamma_plan(nr, nc, b, precision).work_bytes;
}

int ka_gamma_apply(int kernel, double sigma, double ell, const float* xr_dev, int64_t nr, const float* xc_dev,
                   int64_t nc, const float* Y_dev, int b, float* Z_dev, int precision, void* work_dev,
                   size_t work_bytes, void* stream) {
  if (kernel != KA_GAUSSIAN && kernel != KA_EXP_L1) return fail(KA_ERR_ARG, "bad kernel");
  if (precision != KA_FP32 && precision != KA_BF16X3) return fail(KA_ERR_ARG, "bad precision");
  if (b != 16 && b != 32 && b != 64) return fail(KA_ERR_ARG, "b must be 16, 32 or 64");
  if (nr < 0 || nc < 0) return fail(KA_ERR_ARG, "negative size");
  if (!(ell > 0) || !(sigma > 0)) return fail(KA_ERR_ARG, "ell and sigma must be > 0");
  if (nr == 0) return KA_OK;
  if (!xr_dev || !Z_dev || (nc > 0 && (!xc_dev || !Y_dev))) return fail(KA_ERR_ARG, "NULL pointer");
  if (((uintptr_t)Y_dev & 15) != 0) return fail(KA_ERR_ARG, "Y must be 16-byte aligned");
  const GammaPlan gp = gamma_plan(nr, nc, b, precision);
  if (gp.work_bytes > work_bytes || (gp.work_bytes > 0 && !work_dev))
    return fail(KA_ERR_ARG, "workspace too small (see ka_gamma_workspace)");
  if (((uintptr_t)work_dev & 15) != 0) return fail(KA_ERR_ARG, "workspace must be 16-byte aligned");
  GammaLaunch g;
  g.xr = xr_dev;
  g.xr_stride = 3;
  g.rs = nullptr;
  g.nr = nr;
  g.xc = xc_dev;
  g.xc_stride = 3;
  g.nc = nc;
  g.Y = Y_dev;
  g.Z = Z_dev;
  g.partial = (float*)work_dev;
  g.ys = nullptr;   // launch_gamma places it in the workspace
  g.coord_scale = kernel_coord_scale(kernel, ell);
  g.out_scale = (float)(sigma * sigma);
  g.nsplit = 1;
  g.cols_per_split = 0;
  g.row_blocks = 0;
  g.xcd_splits = 0;   // launch_gamma fills the plan
  const hipError_t e = launch_gamma(g, kernel, b, precision, (hipStream_t)stream);
  if (e != hipSuccess) return fail(KA_ERR_HIP, std::string("kernel product launch: ") + hipGetErrorString(e));
  return KA_OK;
}

int ka_profile_enable(ka_problem* p, int on) {
  Problem* P = reinterpret_cast<Problem*>(p);
  if (!P) return fail(KA_ERR_ARG, "problem is NULL");
  P->profile = on != 0;
  return KA_OK;
}

int ka_profile_read(ka_problem* p, int* launches, double* total_ms, double* pairs) {
  Problem* P = reinterpret_cast<Problem*>(p);
  if (!P) return fail(KA_ERR_ARG, "problem is NULL");
  double ms = 0.0;
  for (int i = 0; i < P->prof_launches; ++i) {
    if (hipEventSynchronize(P->ev_stop[i]) != hipSuccess) return fail(KA_ERR_HIP, "event synchronize failed");
    float t = 0.f;
    if (hipEventElapsedTime(&t, P->ev_start[i], P->ev_stop[i]) != hipSuccess)
      return fail(KA_ERR_HIP, "event elapsed time failed");
    ms += t;
  }
  if (launches) *launches = P->prof_launches;
  if (total_ms) *total_ms = ms;
  if (pairs) *pairs = P->prof_pairs;
  return KA_OK;
}

int ka_profile_reset(ka_problem* p) {
  Problem* P = reinterpret_cast<Problem*>(p);
  if (!P) return fail(KA_ERR_ARG, "problem is NULL");
  P->prof_launches = 0;
  P->prof_pairs = 0.0;
  P->prof_ms = 0.0;
  return KA_OK;
}

void ka_destroy(ka_problem* p) { destroy_problem(reinterpret_cast<Problem*>(p)); }

}  // extern "C"
