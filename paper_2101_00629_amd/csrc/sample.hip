// Sampling of the truncated Karhunen-Loeve expansion (paper Sec. 2, eq. kle):
//   alpha_M(x, s) = mu + sum_{i < M} sqrt(lambda_i) phi_i(x) xi_i(s)
// on a tensor grid of parametric points, for draws xi passed in.
//
// phi_i is the eigenfunction with coefficient column i of V in the problem's
// trial space (Galerkin: B-splines over sqrt|det DF|; collocation: the NURBS
// functions, or B_j / W on a general NURBS volume), scaled to unit L^2(D)
// norm (the expansion assumes orthonormal eigenfunctions).  Galerkin:
// int_D phi^2 = v^T Z v exactly, with Z = Z_3 x Z_2 x Z_1 the mass matrix.
// Collocation: int_D phi^2 by the collocation rule's Gauss points.
//
// Device work: Kronecker mode products in FP64 (Z v, or the eigenfunction
// values at the Gauss points; the values at the grid for Phi), fixed-order
// column reductions, and the field product F = mu + Phi diag(sqrt(lambda) /
// ||phi||) Xi on the FP64 matrix cores.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ka_internal.hpp"

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return ka::fail(KA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace ka {

typedef double d4v __attribute__((ext_vector_type(4)));

// Column dot products out[i] = sum_q w[q] A[q + i lda] B[q + i ldb] (w optional),
// in two fixed-order passes: workgroup (c, i) sums chunk c of column i, then
// one thread per column adds the chunk sums in order.
__global__ __launch_bounds__(256) void wdot_partial_kernel(const double* __restrict__ A, int64_t lda,
                                                           const double* __restrict__ B, int64_t ldb,
                                                           const double* __restrict__ w, int64_t Q, int64_t clen,
                                                           double* __restrict__ part) {
  __shared__ double red[256];
  const int i = blockIdx.y;
  const int64_t q0 = (int64_t)blockIdx.x * clen;
  const int64_t q1 = (q0 + clen < Q) ? q0 + clen : Q;
  const double* a = A + (int64_t)i * lda;
  const double* b = B + (int64_t)i * ldb;
  double s = 0.0;
  for (int64_t q = q0 + threadIdx.x; q < q1; q += 256) s += (w ? w[q] : 1.0) * a[q] * b[q];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)i * gridDim.x + blockIdx.x] = red[0];
}

__global__ void wdot_final_kernel(const double* __restrict__ part, int nchunk, int n, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)i * nchunk + c];
  out[i] = s;
}

// XiT[s + k S] = f[k] Xi[k + s ldxi]: the draws scaled and laid out sample-fastest.
__global__ void xi_scale_kernel(const double* __restrict__ Xi, int64_t ldxi, int K, int S,
                                const double* __restrict__ f, double* __restrict__ XiT) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)K * S) return;
  const int s = (int)(id % S), k = (int)(id / S);
  XiT[s + (int64_t)k * S] = f[k] * Xi[k + (int64_t)s * ldxi];
}

// F[p + s ldf] = mu + sum_k Phi[p + k ldp] XiT[s + k S].
//
// v_mfma_f64_16x16x4f64 with A = XiT^T (rows: samples) and B = Phi^T
// (columns: points), so a lane's 16 consecutive points land in consecutive
// addresses.  Operand layout (gfx950): A lane l holds (row l % 16, k = l / 16),
// B lane l holds (k = l / 16, column l % 16), accumulator register r of lane l
// holds (row l / 16 + 4 r, column l % 16).  A workgroup of 2 x 2 waves covers
// kFS samples x kFP points (each wave kU x kT MFMA tiles).  Workgroups
// are dealt to the 8 XCDs round-robin by id; the id mapping gives each XCD
// whole point-tiles (all their sample tiles back to back), so a tile of Phi
// is fetched from HBM into one L2 once.
constexpr int kU = 2, kT = 4;                       // 16 x 16 MFMA tiles per wave: samples x points
constexpr int kFS = 2 * 16 * kU, kFP = 2 * 16 * kT;  // workgroup tile (2 x 2 waves)

__global__ __launch_bounds__(256) void kl_field_kernel(const double* __restrict__ Phi, int64_t ldp, int64_t P,
                                                       const double* __restrict__ XiT, int S, int K, double mu,
                                                       double* __restrict__ F, int64_t ldf, int64_t n_pt, int n_st) {
  const int64_t L = blockIdx.x;
  const int64_t j = L / 8;
  const int64_t pt = (L % 8) + 8 * (j / n_st);
  const int st = (int)(j % n_st);
  if (pt >= n_pt) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t p0 = pt * kFP + (wave & 1) * (16 * kT);
  const int s0 = st * kFS + (wave >> 1) * (16 * kU);
  d4v acc[kU][kT];
#pragma unroll
  for (int u = 0; u < kU; ++u)
#pragma unroll
    for (int t = 0; t < kT; ++t) acc[u][t] = (d4v){0.0, 0.0, 0.0, 0.0};
  // operands of k-step k0 (rows k0 + lk of XiT^T and Phi^T); zero past the edges
  auto load = [&](int k0, double* a, double* b) {
    const int k = k0 + lk;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int s = s0 + 16 * u + li;
      a[u] = (k < K && s < S) ? XiT[s + (int64_t)k * S] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kT; ++t) {
      const int64_t p = p0 + 16 * t + li;
      b[t] = (k < K && p < P) ? Phi[p + (int64_t)k * ldp] : 0.0;
    }
  };
  double a[kU], b[kT];
  load(0, a, b);
  for (int k0 = 0; k0 < K; k0 += 4) {
    // the next step's operands are requested before this step's MFMAs; the
    // scheduling barrier keeps the compiler from sinking the loads
    double an[kU], bn[kT];
    load(k0 + 4, an, bn);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int t = 0; t < kT; ++t) acc[u][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[t], acc[u][t], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < kU; ++u) a[u] = an[u];
#pragma unroll
    for (int t = 0; t < kT; ++t) b[t] = bn[t];
  }
#pragma unroll
  for (int u = 0; u < kU; ++u)
#pragma unroll
    for (int t = 0; t < kT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = s0 + 16 * u + lk + 4 * r;
        const int64_t p = p0 + 16 * t + li;
        if (s < S && p < P) F[p + (int64_t)s * ldf] = mu + acc[u][t][r];
      }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

// Workspace of one call, carved from the problem's kept buffer: sizes are
// collected first (256-byte aligned), then the buffer grows if needed.
struct KlArena {
  std::vector<size_t> off;
  size_t total = 0;
  size_t add(size_t doubles) {
    off.push_back(total);
    total += (std::max<size_t>(doubles, 1) * sizeof(double) + 255) / 256 * 256;
    return off.size() - 1;
  }
};

ModeArgs col_mode(const double* in, int64_t in_ld, double* out, int64_t out_ld, const int dims[3], int mode, int m,
                  const double* mat, int nv) {
  ModeArgs a;
  a.in = in;
  a.in_layout = LAYOUT_COL;
  a.in_ld = in_ld;
  a.out = out;
  a.out_layout = LAYOUT_COL;
  a.out_ld = out_ld;
  for (int k = 0; k < 3; ++k) a.n_in[k] = dims[k];
  a.mode = mode;
  a.m = m;
  a.mat = mat;
  a.matT = nullptr;   // column-major layouts read mat
  a.nv = nv;
  a.out_scale = nullptr;
  return a;
}

// (E_3 x E_2 x E_1) V[:, c0 : c0 + nv] -> out (column-major, ld = m0 m1 m2)
hipError_t kron_eval(const int n[3], const int m[3], double* const E[3], const double* V, int64_t ldv, int nv,
                     double* t1, double* t2, double* out, int64_t ld_out, hipStream_t s) {
  const int d0[3] = {n[0], n[1], n[2]};
  const int d1[3] = {m[0], n[1], n[2]};
  const int d2[3] = {m[0], m[1], n[2]};
  hipError_t e = launch_mode_f64(col_mode(V, ldv, t1, (int64_t)m[0] * n[1] * n[2], d0, 0, m[0], E[0], nv), s);
  if (e == hipSuccess)
    e = launch_mode_f64(col_mode(t1, (int64_t)m[0] * n[1] * n[2], t2, (int64_t)m[0] * m[1] * n[2], d1, 1, m[1], E[1], nv), s);
  if (e == hipSuccess) e = launch_mode_f64(col_mode(t2, (int64_t)m[0] * m[1] * n[2], out, ld_out, d2, 2, m[2], E[2], nv), s);
  return e;
}

std::vector<double> to_rows(const Mat& A) { return A.a; }

}  // namespace

}  // namespace ka

using namespace ka;

extern "C" int ka_kl_sample(ka_problem* p, int M, const double* lambda_host, const double* V_dev, int64_t ldv,
                            const int npts[3], const double* grid_host, int nsamples, const double* xi_dev,
                            int64_t ldxi, double mu, double* field_dev, int64_t ldf, void* stream) {
  Problem* P = reinterpret_cast<Problem*>(p);
  if (!P) return fail(KA_ERR_ARG, "problem is NULL");
  if (!lambda_host || !V_dev || !npts || !grid_host || !xi_dev || !field_dev) return fail(KA_ERR_ARG, "NULL argument");
  if (M < 1 || M > P->N) return fail(KA_ERR_ARG, "M must be in 1..N");
  if (nsamples < 1) return fail(KA_ERR_ARG, "nsamples must be >= 1");
  if (ldv < P->N || ldxi < M) return fail(KA_ERR_ARG, "leading dimension too small");
  if (!std::isfinite(mu)) return fail(KA_ERR_ARG, "mu must be finite");
  for (int i = 0; i < M; ++i)
    if (!(lambda_host[i] >= 0) || !std::isfinite(lambda_host[i])) return fail(KA_ERR_ARG, "eigenvalues must be finite and >= 0");
  int64_t Pts = 1;
  size_t off = 0;
  std::vector<Vec> grid(3);
  for (int k = 0; k < 3; ++k) {
    if (npts[k] < 1 || npts[k] > (1 << 20)) return fail(KA_ERR_ARG, "npts must be in 1..2^20");
    grid[k].assign(grid_host + off, grid_host + off + npts[k]);
    off += npts[k];
    for (double x : grid[k])
      if (!(x >= 0.0 && x <= 1.0)) return fail(KA_ERR_ARG, "grid coordinates must lie in [0, 1]");
    Pts *= npts[k];
  }
  if (Pts > ((int64_t)1 << 34)) return fail(KA_ERR_ARG, "grid too large");
  if (ldf < Pts) return fail(KA_ERR_ARG, "ldf must be >= the number of grid points");
  hipStream_t s = stream ? (hipStream_t)stream : P->stream;
  const ka_desc& d = P->d;
  const bool coll = d.method == KA_COLLOCATION;
  const bool nurbs = d.domain == KA_NURBS;
  const bool dir_weights = coll && !nurbs;   // collocation NURBS factors per direction (closed-form domains)
  const Geometry& geo = P->geo;

  // univariate trial matrices at the grid (and, for collocation, at the Gauss points of the norms)
  std::vector<Mat> Eq(3), Eg(3);
  std::vector<Vec> xq(3), wq(3);
  int n[3], mq[3], mg[3];
  for (int k = 0; k < 3; ++k) {
    const int pk = d.degree[k];
    const Vec& t = P->tsol[k];
    n[k] = P->n[k];
    mg[k] = npts[k];
    mq[k] = n[k];
    if (!trial_matrix_1d(geo, dir_weights, t, pk, k, grid[k], Eg[k]))
      return fail(KA_ERR_SINGULAR, "weight interpolation matrix is singular");
    if (coll && !P->kl_omega) {
      element_gauss(t, d.nq > 0 ? d.nq : pk + 1, xq[k], wq[k]);
      if (!trial_matrix_1d(geo, dir_weights, t, pk, k, xq[k], Eq[k]))
        return fail(KA_ERR_SINGULAR, "weight interpolation matrix is singular");
      mq[k] = (int)xq[k].size();
    } else if (coll) {
      mq[k] = P->kl_mq[k];
    }
  }
  // collocation: weights of int_D phi^2 at the Gauss points, |det DF| (times 1 / W^2 on a NURBS volume)
  const int64_t Q = (int64_t)mq[0] * mq[1] * mq[2];
  std::vector<double> omega;
  if (coll && !P->kl_omega) {
    omega.resize(Q);
    for (int64_t i = 0; i < Q; ++i) {
      const int64_t a1 = i % mq[0], a2 = (i / mq[0]) % mq[1], a3 = i / ((int64_t)mq[0] * mq[1]);
      const double xh[3] = {xq[0][a1], xq[1][a2], xq[2][a3]};
      double x[3], J, W;
      geo.eval(xh, x, &J, &W);
      omega[i] = wq[0][a1] * wq[1][a2] * wq[2][a3] * J / (W * W);
    }
  }
  // per-point scale of phi on the grid: Galerkin 1/sqrt|det DF|, NURBS collocation 1/W
  std::vector<double> gscale;
  if (!coll || nurbs) {
    gscale.resize(Pts);
    for (int64_t i = 0; i < Pts; ++i) {
      const int64_t a1 = i % mg[0], a2 = (i / mg[0]) % mg[1], a3 = i / ((int64_t)mg[0] * mg[1]);
      const double xh[3] = {grid[0][a1], grid[1][a2], grid[2][a3]};
      double x[3], J, W;
      geo.eval(xh, x, &J, &W);
      gscale[i] = coll ? 1.0 / W : 1.0 / std::sqrt(J);
    }
  }

  // collocation norm data: computed on the first call, kept by the problem
  auto keep = [&](const std::vector<double>& v) -> double* {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(double);
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    P->allocs.push_back({p, bytes});
    P->device_bytes += bytes;
    if (hipMemcpy(p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return (double*)p;
  };
  if (coll && !P->kl_omega) {
    for (int k = 0; k < 3; ++k) {
      P->kl_Eq[k] = keep(to_rows(Eq[k]));
      if (!P->kl_Eq[k]) return fail(KA_ERR_OOM, "device allocation failed in ka_kl_sample");
      P->kl_mq[k] = mq[k];
    }
    P->kl_omega = keep(omega);
    if (!P->kl_omega) return fail(KA_ERR_OOM, "device allocation failed in ka_kl_sample");
  }
  // this call's workspace
  const int chunk = std::min(M, 32);
  const int64_t tq = std::max((int64_t)mq[0] * n[1] * n[2], (int64_t)mq[0] * mq[1] * n[2]);
  const int64_t tg = std::max((int64_t)mg[0] * n[1] * n[2], (int64_t)mg[0] * mg[1] * n[2]);
  const int64_t clen = std::max<int64_t>(8192, (Q + 255) / 256);
  const int nchunk = (int)((Q + clen - 1) / clen);
  std::vector<std::vector<double>> Eg_rows(3);
  KlArena ar;
  size_t iEg[3];
  for (int k = 0; k < 3; ++k) {
    Eg_rows[k] = to_rows(Eg[k]);
    iEg[k] = ar.add(Eg_rows[k].size());
  }
  const size_t it1 = ar.add((size_t)std::max(tq, tg) * chunk), it2 = ar.add((size_t)std::max(tq, tg) * chunk);
  const size_t iUq = ar.add((size_t)Q * chunk), ipart = ar.add((size_t)nchunk * chunk), inorm = ar.add(M);
  const size_t iPhi = ar.add((size_t)Pts * M), igs = ar.add(gscale.size()), ifac = ar.add(M);
  const size_t iXi = ar.add((size_t)M * nsamples);
  if (P->kl_bytes < ar.total) {
    if (P->kl_buf) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(P->kl_buf);
      P->kl_buf = nullptr;
      P->kl_bytes = 0;
    }
    if (hipMalloc(&P->kl_buf, ar.total) != hipSuccess) {
      P->kl_buf = nullptr;
      return fail(KA_ERR_OOM, "device allocation failed in ka_kl_sample");
    }
    P->kl_bytes = ar.total;
  }
  auto at = [&](size_t i) { return (double*)((char*)P->kl_buf + ar.off[i]); };
  double* Eqd[3];
  double* Egd[3];
  for (int k = 0; k < 3; ++k) {
    Eqd[k] = coll ? P->kl_Eq[k] : P->Zk[k];   // Galerkin: Z v with the mass matrices
    Egd[k] = at(iEg[k]);
    HIP_TRY(hipMemcpyAsync(Egd[k], Eg_rows[k].data(), Eg_rows[k].size() * sizeof(double), hipMemcpyHostToDevice, s));
  }
  double* t1 = at(it1);
  double* t2 = at(it2);
  double* Uq = at(iUq);
  const double* omega_d = coll ? P->kl_omega : nullptr;
  double* part = at(ipart);
  double* norms2 = at(inorm);
  double* Phi = at(iPhi);
  double* gscale_d = gscale.empty() ? nullptr : at(igs);
  if (gscale_d) HIP_TRY(hipMemcpyAsync(gscale_d, gscale.data(), gscale.size() * sizeof(double), hipMemcpyHostToDevice, s));
  double* fac_d = at(ifac);
  double* XiT = at(iXi);

  for (int c0 = 0; c0 < M; c0 += chunk) {
    const int nv = std::min(chunk, M - c0);
    const double* Vc = V_dev + (int64_t)c0 * ldv;
    // collocation: phi at the Gauss points, norms^2 = sum omega phi^2; Galerkin: Z v, norms^2 = v^T Z v
    HIP_TRY(kron_eval(n, mq, Eqd, Vc, ldv, nv, t1, t2, Uq, Q, s));
    hipLaunchKernelGGL(wdot_partial_kernel, dim3(nchunk, nv), dim3(256), 0, s, Uq, Q, coll ? (const double*)Uq : Vc,
                       coll ? Q : ldv, omega_d, Q, clen, part);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(wdot_final_kernel, dim3((nv + 63) / 64), dim3(64), 0, s, part, nchunk, nv, norms2 + c0);
    HIP_TRY(hipGetLastError());
    HIP_TRY(kron_eval(n, mg, Egd, Vc, ldv, nv, t1, t2, Phi + (int64_t)c0 * Pts, Pts, s));
  }
  if (gscale_d) HIP_TRY(scale_rows(Phi, Pts, M, Pts, gscale_d, s));
  std::vector<double> nrm(M), fac(M);
  HIP_TRY(hipMemcpyAsync(nrm.data(), norms2, M * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < M; ++i) {
    if (!(nrm[i] > 0) || !std::isfinite(nrm[i])) return fail(KA_ERR_SINGULAR, "an eigenfunction has zero L2 norm");
    fac[i] = std::sqrt(lambda_host[i] / nrm[i]);
  }
  HIP_TRY(hipMemcpyAsync(fac_d, fac.data(), M * sizeof(double), hipMemcpyHostToDevice, s));
  const int64_t tot = (int64_t)M * nsamples;
  hipLaunchKernelGGL(xi_scale_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, xi_dev, ldxi, M, nsamples,
                     fac_d, XiT);
  HIP_TRY(hipGetLastError());
  const int64_t n_pt = (Pts + kFP - 1) / kFP;
  const int n_st = (nsamples + kFS - 1) / kFS;
  const int64_t grid_wg = 8 * ((n_pt + 7) / 8) * (int64_t)n_st;
  if (grid_wg > ((int64_t)1 << 31) - 1) return fail(KA_ERR_ARG, "field too large for one launch");
  hipLaunchKernelGGL(kl_field_kernel, dim3((unsigned)grid_wg), dim3(256), 0, s, Phi, Pts, Pts, XiT, nsamples, M, mu,
                     field_dev, ldf, n_pt, n_st);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));   // the host vectors copied above live until here
  return KA_OK;
}
