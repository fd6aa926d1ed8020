// Kronecker mode products: the "linear or nearly linear" steps of both
// matrix-free operators (paper Sec. 3.1: L^-T, M, B~^-T, J and their
// transposes; Sec. 3.2 / Algorithm 1: R at the quadrature points, J W
// scaling, the LU backsolve of Z).  A Kronecker matrix A3 (x) A2 (x) A1 acts
// on a block as three mode products, each contracting one tensor index with
// a small dense univariate matrix.
//
// One thread per output element; threads are ordered like the output's
// memory so the stores coalesce.  The univariate matrix (at most a few
// hundred rows) is read through the cache.
#include <hip/hip_runtime.h>

#include "ka_internal.hpp"

namespace ka {

template <typename TIn, typename TAcc, typename TOut>
__global__ void mode_product_kernel(ModeArgs a, int64_t total) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  int no[3] = {a.n_in[0], a.n_in[1], a.n_in[2]};
  no[a.mode] = a.m;
  const int64_t Nout = (int64_t)no[0] * no[1] * no[2];
  int64_t i, j;
  // Threads follow the input's memory order, so the reads coalesce; when the
  // output layout differs, the scattered stores of a workgroup fill whole
  // lines in the write-back L2 before they reach HBM.  (Following the
  // output's order instead made every input read stride over whole point
  // rows: 19 ms instead of about 1 ms for a 287,496 x 64 point-major FP32 to
  // column-major FP64 product.)
  if (a.in_layout == LAYOUT_COL) { i = id % Nout; j = id / Nout; }
  else { i = id / a.nv; j = id % a.nv; }   // threads over the nv live columns
  const int o1 = (int)(i % no[0]);
  const int o2 = (int)((i / no[0]) % no[1]);
  const int o3 = (int)(i / ((int64_t)no[0] * no[1]));
  const int o[3] = {o1, o2, o3};
  const int64_t stride_in[3] = {1, a.n_in[0], (int64_t)a.n_in[0] * a.n_in[1]};
  int oi[3] = {o1, o2, o3};
  oi[a.mode] = 0;
  const int64_t base = oi[0] + (int64_t)a.n_in[0] * (oi[1] + (int64_t)a.n_in[1] * oi[2]);
  const int nk = a.n_in[a.mode];
  const TAcc* mrow = reinterpret_cast<const TAcc*>(a.mat) + (int64_t)o[a.mode] * nk;
  const TIn* in = reinterpret_cast<const TIn*>(a.in);
  TAcc s = 0;
  if (a.in_layout == LAYOUT_COL) {
    const TIn* src = in + base + j * a.in_ld;
    const int64_t st = stride_in[a.mode];
    for (int c = 0; c < nk; ++c) s += mrow[c] * (TAcc)src[c * st];
  } else {
    const TIn* src = in + base * a.in_ld + j;
    const int64_t st = stride_in[a.mode] * a.in_ld;
    for (int c = 0; c < nk; ++c) s += mrow[c] * (TAcc)src[c * st];
  }
  if (a.out_scale) s *= (TAcc)a.out_scale[i];
  TOut* out = reinterpret_cast<TOut*>(a.out);
  if (a.out_layout == LAYOUT_COL) out[i + j * a.out_ld] = (TOut)s;
  else out[i * a.out_ld + j] = (TOut)s;
}

template <typename TIn, typename TAcc, typename TOut>
static hipError_t launch_mode(const ModeArgs& a, hipStream_t s) {
  int no[3] = {a.n_in[0], a.n_in[1], a.n_in[2]};
  no[a.mode] = a.m;
  const int64_t total = (int64_t)no[0] * no[1] * no[2] * a.nv;
  if (total == 0) return hipSuccess;
  const int threads = 256;
  hipLaunchKernelGGL((mode_product_kernel<TIn, TAcc, TOut>), dim3((unsigned)((total + threads - 1) / threads)),
                     dim3(threads), 0, s, a, total);
  return hipGetLastError();
}

hipError_t launch_mode_f64(const ModeArgs& a, hipStream_t s) { return launch_mode<double, double, double>(a, s); }
hipError_t launch_mode_f64_to_f32(const ModeArgs& a, hipStream_t s) { return launch_mode<double, float, float>(a, s); }
hipError_t launch_mode_f32(const ModeArgs& a, hipStream_t s) { return launch_mode<float, float, float>(a, s); }
hipError_t launch_mode_f32_to_f64(const ModeArgs& a, hipStream_t s) { return launch_mode<float, float, double>(a, s); }
hipError_t launch_mode_f32in_f64(const ModeArgs& a, hipStream_t s) { return launch_mode<float, double, double>(a, s); }

__global__ void cast_pt32_col64_kernel(const float* __restrict__ in, int64_t ld_in, double* __restrict__ out,
                                       int64_t ld_out, int64_t npts, int nv, const double* __restrict__ div) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= npts * nv) return;
  const int64_t i = id % npts, j = id / npts;
  const double v = (double)in[i * ld_in + j];
  out[i + j * ld_out] = div ? v / div[i] : v;
}

hipError_t cast_pt32_to_col64(const float* in, int64_t ld_in, double* out, int64_t ld_out, int64_t npts, int nv,
                              const double* div, hipStream_t s) {
  const int64_t tot = npts * nv;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(cast_pt32_col64_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, in, ld_in, out,
                     ld_out, npts, nv, div);
  return hipGetLastError();
}

}  // namespace ka
