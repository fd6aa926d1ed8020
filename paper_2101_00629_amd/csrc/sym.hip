// Device driver of the small symmetric eigensolve (sym_core.hpp) used by the
// Galerkin Rayleigh-Ritz step: the tridiagonalisation runs as one workgroup
// (working matrix in LDS up to order 128), the other stages as grids with one
// wave per eigenvalue, one thread per cluster and one thread per vector; only
// the leading nvec eigenvectors are formed.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ka_internal.hpp"
#include "sym_core.hpp"

namespace ka {

constexpr int kTriThreads = 512;
constexpr int kTriLds = 128;
constexpr int kSymTriMax = 1024;
constexpr int kTriNb = kSymNbMax;   // panel width of the blocked reduction
constexpr int kBackLds = 240;

size_t sym_tri_work(int n) { return sym_tri_work_doubles(n); }

struct BlockTeam {
  double* red;    // one slot per wave
  double* redv;   // kVecMax slots per wave (sumv)
  static constexpr int kVecMax = 2 * kSymNbMax;
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
  // out[i] = sum over the workgroup of x[i], i < k <= kVecMax (out: shared)
  __device__ void sumv(const double* x, int k, double* out) const {
#pragma unroll
    for (int i = 0; i < kVecMax; ++i) {
      if (i < k) {
        double y = x[i];
        for (int off = 32; off > 0; off >>= 1) y += __shfl_xor(y, off);
        if ((threadIdx.x & 63) == 0) redv[(threadIdx.x >> 6) * kVecMax + i] = y;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kTriThreads / 64; ++w) s += redv[w * kVecMax + threadIdx.x];
      out[threadIdx.x] = s;
    }
    __syncthreads();
  }
};

template <bool LDS>
__global__ __launch_bounds__(kTriThreads) void sym_tridiag_kernel(const double* __restrict__ H, int n, int ldh,
                                                                  double* __restrict__ work) {
  __shared__ double A_lds[LDS ? kTriLds * kTriLds : 1];
  __shared__ double v[kSymTriMax], w[kSymTriMax];
  __shared__ double red[kTriThreads / 64];
  // blocked reduction (matrix in device memory): the panel's V and W columns
  __shared__ double VW[LDS ? 1 : 2 * kSymTriMax * kSymNbMax];
  __shared__ double yz[BlockTeam::kVecMax], redv[(kTriThreads / 64) * BlockTeam::kVecMax];
  const SymWork sw = sym_work_split(work, n);
  double* A = LDS ? A_lds : sw.A;
  for (int j = 0; j < n; ++j)
    for (int i = threadIdx.x; i < n; i += kTriThreads)
      A[i + (int64_t)j * n] = 0.5 * (H[i + (int64_t)j * ldh] + H[j + (int64_t)i * ldh]);
  __syncthreads();
  BlockTeam tm{red, redv};
  if constexpr (LDS)
    sym_tridiagonalize(tm, A, n, sw.d, sw.e, sw.beta, v, w);
  else
    sym_tridiagonalize_blocked(tm, A, n, sw.d, sw.e, sw.beta, v, w, VW, VW + (size_t)n * kSymNbMax, yz, kTriNb);
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

// one thread per cluster that meets the wanted range [n - nvec, n).  Up to
// order MAXN a workgroup of NT threads keeps each thread's LU fields and
// iterated vector in LDS ([field][i][thread]; 6 MAXN NT doubles): 16 threads
// up to order 200, 2 up to 512, 1 up to 960.  Above that they live in the
// interleaved global arrays F and Xw (64 threads per workgroup).
template <bool LDS, int NT, int MAXN>
__global__ __launch_bounds__(NT) void sym_invit_kernel(double* __restrict__ work, int n, int nvec) {
  __shared__ double sd[LDS ? MAXN : kSymTriMax], se[LDS ? MAXN : kSymTriMax];
  __shared__ double fx[LDS ? 6 * MAXN * NT : 1];
  const SymWork sw = sym_work_split(work, n);
  for (int i = threadIdx.x; i < n; i += NT) {
    sd[i] = sw.d[i];
    se[i] = (i + 1 < n) ? sw.e[i] : 0.0;
  }
  __syncthreads();
  const int t = threadIdx.x;
  const int k = n - nvec + blockIdx.x * NT + t;
  if (k < n && sym_cluster_top(sw.lam, n, k, sw.bnd)) {
    if (LDS)
      sym_inverse_iteration(sd, se, n, sw.lam, k, n - nvec, sw.bnd, sw.V, fx + t, (size_t)n * NT, NT,
                            fx + 5 * (size_t)n * NT + t, NT);
    else
      sym_inverse_iteration(sd, se, n, sw.lam, k, n - nvec, sw.bnd, sw.V, sw.F + k, (size_t)n * n, n, sw.Xw + k, n);
  }
}

// one thread per wanted vector; the workgroup's 64 vectors are staged in LDS
// (element i of vector t at xs[i * 64 + t]) up to order kBackLds

template <bool LDS>
__global__ __launch_bounds__(64) void sym_back_kernel(double* __restrict__ work, int n, int nvec) {
  __shared__ double xs[LDS ? kBackLds * 64 : 1];
  __shared__ double vs[kSymTriMax];
  const SymWork sw = sym_work_split(work, n);
  const int t = threadIdx.x;
  const int k = n - nvec + blockIdx.x * 64 + t;
  const bool act = k < n;
  double* x = LDS ? xs + t : sw.V + (act ? k : 0);
  const int stride = LDS ? 64 : n;
  if (LDS)
    for (int i = 0; i < n; ++i) xs[i * 64 + t] = act ? sw.V[(int64_t)i * n + k] : 0.0;
  for (int j = n - 3; j >= 0; --j) {
    const double b = sw.beta[j];
    if (b == 0.0) continue;                      // uniform over the workgroup
    const int m = n - j - 1;
    __syncthreads();
    for (int i = t; i < m; i += 64) vs[i] = sw.A[(j + 1 + i) + (int64_t)j * n];
    __syncthreads();
    if (LDS || act) sym_reflect(vs, m, b, x + (size_t)(j + 1) * stride, stride);
  }
  if (LDS && act)
    for (int i = 0; i < n; ++i) sw.V[(int64_t)i * n + k] = xs[i * 64 + t];
}

// Above order kBackLds: one wave per 4 vectors, 16 lanes per vector.  Lane r
// of a vector holds its elements r, r + 16, ... (NS of them) in registers;
// for each reflector the 16 lanes form the dot product with a fixed
// butterfly, then update their own elements.  No barriers: every wave walks
// the reflectors (read through the cache) on its own.
template <int NS>
__global__ __launch_bounds__(64) void sym_back_wave_kernel(double* __restrict__ work, int n, int nvec) {
  const SymWork sw = sym_work_split(work, n);
  const int lane = threadIdx.x & 63, r = lane & 15;
  const int k = n - nvec + blockIdx.x * 4 + (lane >> 4);
  const bool act = k < n;
  const int kk = act ? k : n - 1;
  double x[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = r + 16 * s;
    x[s] = (i < n) ? sw.V[(int64_t)i * n + kk] : 0.0;
  }
  for (int j = n - 3; j >= 0; --j) {
    const double b = sw.beta[j];
    if (b == 0.0) continue;                      // uniform over the grid
    const double* v = sw.A + (int64_t)j * n;     // reflector: rows j + 1 .. n - 1 of column j
    double dot = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = r + 16 * s;
      if (i > j && i < n) dot += v[i] * x[s];
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 16);
    const double sc = b * dot;
#pragma unroll
    for (int s = 0; s < NS; ++s) {          // v again, now from the cache
      const int i = r + 16 * s;
      if (i > j && i < n) x[s] -= sc * v[i];
    }
  }
  if (act)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = r + 16 * s;
      if (i < n) sw.V[(int64_t)i * n + k] = x[s];
    }
}

// theta descending (all n); S column k (k < nvec) = vector n-1-k
__global__ __launch_bounds__(256) void sym_out_kernel(const double* __restrict__ work, int n, int nvec,
                                                      double* __restrict__ theta, double* __restrict__ S, int lds) {
  const SymWork sw = sym_work_split(const_cast<double*>(work), n);
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q < n) theta[q] = sw.lam[n - 1 - q];
  if (q >= (int64_t)n * nvec) return;
  const int i = (int)(q % n), k = (int)(q / n);
  S[i + (int64_t)k * lds] = sw.V[(int64_t)i * n + (n - 1 - k)];
}

hipError_t sym_eig_tri(const double* H, int n, int ldh, int nvec, double* theta, double* S, int lds, double* work,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > kSymTriMax || ldh < n || lds < n || nvec < 0 || nvec > n) return hipErrorInvalidValue;
  if (n <= kTriLds)
    hipLaunchKernelGGL(sym_tridiag_kernel<true>, dim3(1), dim3(kTriThreads), 0, s, H, n, ldh, work);
  else
    hipLaunchKernelGGL(sym_tridiag_kernel<false>, dim3(1), dim3(kTriThreads), 0, s, H, n, ldh, work);
  hipLaunchKernelGGL(sym_section_kernel, dim3(n), dim3(64), 0, s, work, n);
  if (nvec > 0) {
    const int g64 = (nvec + 63) / 64;
    if (n <= 200)
      hipLaunchKernelGGL((sym_invit_kernel<true, 16, 200>), dim3((nvec + 15) / 16), dim3(16), 0, s, work, n, nvec);
    else if (n <= 512)
      hipLaunchKernelGGL((sym_invit_kernel<true, 2, 512>), dim3((nvec + 1) / 2), dim3(2), 0, s, work, n, nvec);
    else if (n <= 960)
      hipLaunchKernelGGL((sym_invit_kernel<true, 1, 960>), dim3(nvec), dim3(1), 0, s, work, n, nvec);
    else
      hipLaunchKernelGGL((sym_invit_kernel<false, 64, 1>), dim3(g64), dim3(64), 0, s, work, n, nvec);
    const int g4 = (nvec + 3) / 4;
    if (n <= kBackLds)
      hipLaunchKernelGGL(sym_back_kernel<true>, dim3(g64), dim3(64), 0, s, work, n, nvec);
    else if (n <= 512)
      hipLaunchKernelGGL(sym_back_wave_kernel<32>, dim3(g4), dim3(64), 0, s, work, n, nvec);
    else
      hipLaunchKernelGGL(sym_back_wave_kernel<64>, dim3(g4), dim3(64), 0, s, work, n, nvec);
  }
  const int64_t nq = std::max<int64_t>((int64_t)n * nvec, n);
  hipLaunchKernelGGL(sym_out_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, work, n, nvec, theta, S,
                     lds);
  return hipGetLastError();
}

}  // namespace ka
