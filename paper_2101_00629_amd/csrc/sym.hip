// Device driver of the small symmetric eigensolve (sym_core.hpp) used by the
// Galerkin Rayleigh-Ritz step: the tridiagonalisation runs as one workgroup
// (working matrix in LDS up to order 128), the other stages as grids with one
// wave per eigenvalue, one thread per cluster and one thread per vector.
#include <hip/hip_runtime.h>

#include "ka_internal.hpp"
#include "sym_core.hpp"

namespace ka {

constexpr int kTriThreads = 512;
constexpr int kTriLds = 128;
constexpr int kSymTriMax = 1024;

size_t sym_tri_work(int n) { return sym_tri_work_doubles(n); }

struct BlockTeam {
  double* red;   // one slot per wave
  __device__ int tid() const { return threadIdx.x; }
  __device__ int size() const { return kTriThreads; }
  __device__ void sync() const { __syncthreads(); }
  __device__ double sum(double x) const {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kTriThreads / 64; ++w) s += red[w];
    __syncthreads();
    return s;
  }
};

template <bool LDS>
__global__ __launch_bounds__(kTriThreads) void sym_tridiag_kernel(const double* __restrict__ H, int n, int ldh,
                                                                  double* __restrict__ work) {
  __shared__ double A_lds[LDS ? kTriLds * kTriLds : 1];
  __shared__ double v[kSymTriMax], w[kSymTriMax];
  __shared__ double red[kTriThreads / 64];
  const SymWork sw = sym_work_split(work, n);
  double* A = LDS ? A_lds : sw.A;
  for (int64_t q = threadIdx.x; q < (int64_t)n * n; q += kTriThreads) {
    const int i = (int)(q % n), j = (int)(q / n);
    A[q] = 0.5 * (H[i + (int64_t)j * ldh] + H[j + (int64_t)i * ldh]);
  }
  __syncthreads();
  BlockTeam tm{red};
  sym_tridiagonalize(tm, A, n, sw.d, sw.e, sw.beta, v, w);
  if (LDS)
    for (int64_t q = threadIdx.x; q < (int64_t)n * n; q += kTriThreads) sw.A[q] = A[q];
  if (threadIdx.x == 0) sym_bounds(sw.d, sw.e, n, sw.bnd);
}

// one wave per eigenvalue: 64-point multisection
__global__ __launch_bounds__(64) void sym_section_kernel(double* __restrict__ work, int n) {
  __shared__ double sd[kSymTriMax], se[kSymTriMax];
  const SymWork sw = sym_work_split(work, n);
  const int t = threadIdx.x;
  for (int i = t; i < n; i += 64) {
    sd[i] = sw.d[i];
    se[i] = (i + 1 < n) ? sw.e[i] : 0.0;
  }
  __syncthreads();
  const int k = blockIdx.x;
  const double pivmin = sym_pivmin(sw.bnd);
  double lo = sw.bnd[0], hi = sw.bnd[1];
  for (int r = 0; r < kSymSectionRounds && !sym_section_done(lo, hi, sw.bnd); ++r) {
    const int c = sym_sturm_count(sd, se, n, sym_section_point(lo, hi, t, 64), pivmin);
    const uint64_t mask = __ballot(c > k);
    sym_section_narrow(lo, hi, mask, 64);
  }
  if (t == 0) sw.lam[k] = 0.5 * (lo + hi);
}

// one thread per cluster of eigenvalues
__global__ __launch_bounds__(64) void sym_invit_kernel(double* __restrict__ work, int n) {
  __shared__ double sd[kSymTriMax], se[kSymTriMax];
  const SymWork sw = sym_work_split(work, n);
  for (int i = threadIdx.x; i < n; i += 64) {
    sd[i] = sw.d[i];
    se[i] = (i + 1 < n) ? sw.e[i] : 0.0;
  }
  __syncthreads();
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k < n && sym_cluster_start(sw.lam, k, sw.bnd)) sym_inverse_iteration(sd, se, n, sw.lam, k, sw.bnd, sw.V, sw.F);
}

// one thread per vector
__global__ __launch_bounds__(64) void sym_back_kernel(double* __restrict__ work, int n) {
  const SymWork sw = sym_work_split(work, n);
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k < n) sym_back_transform(sw.A, sw.beta, n, sw.V, k);
}

// theta descending, S column k = vector n-1-k
__global__ __launch_bounds__(256) void sym_out_kernel(const double* __restrict__ work, int n,
                                                      double* __restrict__ theta, double* __restrict__ S, int lds) {
  const SymWork sw = sym_work_split(const_cast<double*>(work), n);
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (int64_t)n * n) return;
  const int i = (int)(q % n), k = (int)(q / n);
  const int src = n - 1 - k;
  S[i + (int64_t)k * lds] = sw.V[(int64_t)i * n + src];
  if (i == 0) theta[k] = sw.lam[src];
}

hipError_t sym_eig_tri(const double* H, int n, int ldh, double* theta, double* S, int lds, double* work,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > kSymTriMax || ldh < n || lds < n) return hipErrorInvalidValue;
  if (n <= kTriLds)
    hipLaunchKernelGGL(sym_tridiag_kernel<true>, dim3(1), dim3(kTriThreads), 0, s, H, n, ldh, work);
  else
    hipLaunchKernelGGL(sym_tridiag_kernel<false>, dim3(1), dim3(kTriThreads), 0, s, H, n, ldh, work);
  const int g64 = (n + 63) / 64;
  hipLaunchKernelGGL(sym_section_kernel, dim3(n), dim3(64), 0, s, work, n);
  hipLaunchKernelGGL(sym_invit_kernel, dim3(g64), dim3(64), 0, s, work, n);
  hipLaunchKernelGGL(sym_back_kernel, dim3(g64), dim3(64), 0, s, work, n);
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(sym_out_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, work, n, theta, S, lds);
  return hipGetLastError();
}

}  // namespace ka
