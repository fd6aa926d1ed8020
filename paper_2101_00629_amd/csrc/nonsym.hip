// Device wrapper of the small non-symmetric eigensolve (nonsym_core.hpp):
// one workgroup of a single wave, so every team synchronisation is a cheap
// one-wave barrier.
#include <hip/hip_runtime.h>

#include "ka_internal.hpp"
#include "nonsym_core.hpp"

namespace ka {

constexpr int kNsThreads = 64;
constexpr int kNsMax = 1024;

size_t nonsym_eig_work(int n) { return nonsym_work_doubles(n); }

struct WaveTeam {
  double* scratch;
  __device__ int tid() const { return threadIdx.x; }
  __device__ int size() const { return kNsThreads; }
  __device__ void sync() const { __syncthreads(); }
  __device__ double sum(double x) const {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
  }
};

constexpr int kNsLds = 120;   // working matrix in LDS up to this order (112.5 KB)

template <bool LDS>
__global__ __launch_bounds__(kNsThreads) void nonsym_eig_kernel(const double* __restrict__ H, int n, int ldh,
                                                                double* __restrict__ wr, double* __restrict__ wi,
                                                                double* __restrict__ S, int lds,
                                                                double* __restrict__ work, int* status) {
  // team scratch: Householder vector (n) and the per-sweep log (6n)
  __shared__ double v[LDS ? 6 * kNsLds : 6 * kNsMax];
  __shared__ double A_lds[LDS ? kNsLds * kNsLds : 1];
  WaveTeam tm{v};
  nonsym_core(tm, H, n, ldh, wr, wi, S, lds, work, status, LDS ? A_lds : nullptr);
}

hipError_t nonsym_eig(const double* H, int n, int ldh, double* wr, double* wi, double* S, int lds, double* work,
                      int* status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > kNsMax) return hipErrorInvalidValue;
  if (n <= kNsLds)
    hipLaunchKernelGGL(nonsym_eig_kernel<true>, dim3(1), dim3(kNsThreads), 0, s, H, n, ldh, wr, wi, S, lds, work,
                       status);
  else
    hipLaunchKernelGGL(nonsym_eig_kernel<false>, dim3(1), dim3(kNsThreads), 0, s, H, n, ldh, wr, wi, S, lds, work,
                       status);
  return hipGetLastError();
}

}  // namespace ka
