// Device driver of the small non-symmetric eigensolve (nonsym_core.hpp) used
// by the collocation Rayleigh-Ritz step: Hessenberg reduction by one
// workgroup (matrix in LDS up to order 128), eigenvalue QR by one wave on a
// banded copy (LDS up to order 192), then grids for ranking, inverse
// iteration (one wave per cluster of wanted eigenvalues), back-
// transformation (one thread per wanted column) and output.
#include <hip/hip_runtime.h>

#include "ka_internal.hpp"
#include "nonsym_core.hpp"

namespace ka {

constexpr int kNsThreads = 512;
constexpr int kNsHessLds = 128;
constexpr int kNsBandLds = 192;
constexpr int kNsMax = 1024;
constexpr int kNsBackLds = 240;
constexpr int kNsInvLds = 128;

size_t nonsym_eig_work(int n, int nvec_max) {
  const int nv = nvec_max + 1 < n ? nvec_max + 1 : n;
  return nonsym_work_doubles(n, nv);
}

static int ns_stride(int n, int nvec) { return nvec + 1 < n ? nvec + 1 : n; }

template <int NT>
struct NsTeam {
  double* red;
  __device__ int tid() const { return threadIdx.x; }
  __device__ int size() const { return NT; }
  __device__ void sync() const { __syncthreads(); }
  __device__ double sum(double x) const {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if (NT == 64) return x;
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    __syncthreads();
    return s;
  }
};

template <bool LDS>
__global__ __launch_bounds__(kNsThreads) void ns_hess_kernel(const double* __restrict__ H, int n, int ldh,
                                                             double* __restrict__ work, int nv) {
  __shared__ double A_lds[LDS ? kNsHessLds * (kNsHessLds + 1) : 1];
  __shared__ double v[kNsMax], w[kNsMax];
  __shared__ double red[kNsThreads / 64];
  const NsWork ws = ns_work_split(work, n, nv);
  const int ld = LDS ? n + 1 : n;
  double* A = LDS ? A_lds : ws.A;
  for (int j = 0; j < n; ++j)
    for (int i = threadIdx.x; i < n; i += kNsThreads) A[i + (size_t)j * ld] = H[i + (int64_t)j * ldh];
  __syncthreads();
  NsTeam<kNsThreads> tm{red};
  ns_hessenberg(tm, A, ld, n, ws.hsub, ws.beta, v, w);
  if (LDS)
    for (int j = 0; j < n; ++j)
      for (int i = threadIdx.x; i < n; i += kNsThreads) ws.A[i + (size_t)j * n] = A[i + (size_t)j * ld];
}

template <bool LDS>
__global__ __launch_bounds__(64) void ns_qr_kernel(double* __restrict__ work, int n, int nv) {
  __shared__ double hb_lds[LDS ? (size_t)kNsBandLds * (kNsBandLds + 7) / 2 + 8 : 1];
  const NsWork ws = ns_work_split(work, n, nv);
  double* hb = LDS ? hb_lds : ws.HB;
  NsTeam<64> tm{nullptr};
  ns_band_fill(tm, ws.A, n, ws.hsub, n, hb, ws.HT);
  __syncthreads();
  const int fail = ns_qr_values(tm, hb, n, ws.wr0, ws.wi0, ws.misc);
  if (threadIdx.x == 0) ws.misc[1] = fail;
}

__global__ __launch_bounds__(256) void ns_rank_kernel(double* __restrict__ work, int n, int nv) {
  const NsWork ws = ns_work_split(work, n, nv);
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  const int r = ns_rank(ws.wr0, n, c);
  ws.wr[r] = ws.wr0[c];
  ws.wi[r] = ws.wi0[c];
}

// one workgroup (one wave) per wanted entry that starts a cluster; the LU
// planes live in LDS up to order kNsInvLds, else in the entry's slot of F
template <bool LDS>
__global__ __launch_bounds__(64) void ns_invit_kernel(double* __restrict__ work, int n, int nv, int nvec) {
  __shared__ double lu_lds[LDS ? kNsInvLds * (kNsInvLds + 1) + 3 * kNsInvLds : 1];
  __shared__ double xs[2 * kNsMax];
  const NsWork ws = ns_work_split(work, n, nv);
  const int c = blockIdx.x;
  const int nw = ns_wanted(ws.wi, n, nvec);
  if (c >= nw || !ns_is_entry(ws.wi, c)) return;
  const double scale = ns_scale(ws.wr, ws.wi, n);
  if (!ns_cluster_first(ws.wr, ws.wi, c, kNsClusterGap * scale)) return;
  double* base = LDS ? lu_lds : ws.F + (size_t)c * ns_lu_doubles(n);
  const size_t plane = ns_lu_plane(n);
  NsTeam<64> tm{nullptr};
  ns_invit_team(tm, ws.HT, ws.hsub, n, ws.wr, ws.wi, c, nw, nv, scale, ws.V, base, base + plane, base + 2 * plane,
                xs);
}

// one thread per wanted column (real and imaginary parts are separate columns)
template <bool LDS>
__global__ __launch_bounds__(64) void ns_back_kernel(double* __restrict__ work, int n, int nv, int nvec) {
  __shared__ double xs[LDS ? kNsBackLds * 64 : 1];
  __shared__ double vs[kNsMax];
  const NsWork ws = ns_work_split(work, n, nv);
  const int t = threadIdx.x;
  const int c = blockIdx.x * 64 + t;
  const bool act = c < ns_wanted(ws.wi, n, nvec);
  double* x = LDS ? xs + t : ws.V + (act ? c : 0);
  const int stride = LDS ? 64 : nv;
  if (LDS)
    for (int i = 0; i < n; ++i) xs[i * 64 + t] = act ? ws.V[(int64_t)i * nv + c] : 0.0;
  for (int j = n - 3; j >= 0; --j) {
    const double b = ws.beta[j];
    if (b == 0.0) continue;                      // uniform over the workgroup
    const int m = n - j - 1;
    __syncthreads();
    for (int i = t; i < m; i += 64) vs[i] = ws.A[(j + 1 + i) + (int64_t)j * n];
    __syncthreads();
    if (LDS || act) sym_reflect(vs, m, b, x + (size_t)(j + 1) * stride, stride);
  }
  if (LDS && act)
    for (int i = 0; i < n; ++i) ws.V[(int64_t)i * nv + c] = xs[i * 64 + t];
}

// eigenvalues (all n, sorted) and the wanted columns, normalised
__global__ __launch_bounds__(256) void ns_out_kernel(const double* __restrict__ work, int n, int nv, int nvec,
                                                     double* __restrict__ wr, double* __restrict__ wi,
                                                     double* __restrict__ S, int lds, int* status) {
  const NsWork ws = ns_work_split(const_cast<double*>(work), n, nv);
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c == 0) *status = (int)ws.misc[1];
  if (c >= n) return;
  wr[c] = ws.wr[c];
  wi[c] = ws.wi[c];
  if (c >= ns_wanted(ws.wi, n, nvec)) return;
  // columns of one pair share a norm
  const bool first = ns_is_entry(ws.wi, c);
  const int c0 = first ? c : c - 1;
  const bool pair = ws.wi[c0] > 0.0;
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    const double a = ws.V[(int64_t)i * nv + c0];
    s += a * a;
    if (pair) {
      const double b = ws.V[(int64_t)i * nv + c0 + 1];
      s += b * b;
    }
  }
  const double sc = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int i = 0; i < n; ++i) S[i + (int64_t)c * lds] = ws.V[(int64_t)i * nv + c] * sc;
}

hipError_t nonsym_eig(const double* H, int n, int ldh, int nvec, double* wr, double* wi, double* S, int lds,
                      double* work, int* status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > kNsMax || ldh < n || lds < n || nvec < 0 || nvec > n) return hipErrorInvalidValue;
  const int nv = ns_stride(n, nvec);
  if (n <= kNsHessLds)
    hipLaunchKernelGGL(ns_hess_kernel<true>, dim3(1), dim3(kNsThreads), 0, s, H, n, ldh, work, nv);
  else
    hipLaunchKernelGGL(ns_hess_kernel<false>, dim3(1), dim3(kNsThreads), 0, s, H, n, ldh, work, nv);
  if (n <= kNsBandLds)
    hipLaunchKernelGGL(ns_qr_kernel<true>, dim3(1), dim3(64), 0, s, work, n, nv);
  else
    hipLaunchKernelGGL(ns_qr_kernel<false>, dim3(1), dim3(64), 0, s, work, n, nv);
  hipLaunchKernelGGL(ns_rank_kernel, dim3((n + 255) / 256), dim3(256), 0, s, work, n, nv);
  const int g64 = (nv + 63) / 64;
  if (nvec > 0) {
    if (n <= kNsInvLds)
      hipLaunchKernelGGL(ns_invit_kernel<true>, dim3(nv), dim3(64), 0, s, work, n, nv, nvec);
    else
      hipLaunchKernelGGL(ns_invit_kernel<false>, dim3(nv), dim3(64), 0, s, work, n, nv, nvec);
    if (n <= kNsBackLds)
      hipLaunchKernelGGL(ns_back_kernel<true>, dim3(g64), dim3(64), 0, s, work, n, nv, nvec);
    else
      hipLaunchKernelGGL(ns_back_kernel<false>, dim3(g64), dim3(64), 0, s, work, n, nv, nvec);
  }
  hipLaunchKernelGGL(ns_out_kernel, dim3((n + 255) / 256), dim3(256), 0, s, work, n, nv, nvec, wr, wi, S, lds,
                     status);
  return hipGetLastError();
}

}  // namespace ka
