// Kronecker mode products: the "linear or nearly linear" steps of both
// matrix-free operators (paper Sec. 3.1: L^-T, M, B~^-T, J and their
// transposes; Sec. 3.2 / Algorithm 1: R at the quadrature points, J W
// scaling, the LU backsolve of Z).  A Kronecker matrix A3 (x) A2 (x) A1 acts
// on a block as three mode products, each contracting one tensor index with
// a small dense univariate matrix.
//
// The operator keeps its blocks point-major (the nv values of a point
// contiguous) between the two ends of a block application, which convert
// from and to the column-major API layout with LDS-tiled transposes.  In the
// point-major layout every mode product reads and writes whole point rows:
// lanes run over the block's vectors, each thread accumulates R outputs
// along the mode from one pass over its input fiber (R-fold reuse of every
// load), and the matrix entries are the same for the whole wave (scalar
// loads).  A general per-output kernel covers the column-major cases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "ka_internal.hpp"

namespace ka {

// Point-major mode product: out[(p_out) * out_ld + j] = scale[p_out] *
// sum_c mat[m * nk + c] * in[(p_in(c)) * in_ld + j], with the matrix given
// transposed (matT[c * m_out + m]) so that the R entries a thread needs per
// input value are contiguous.  Threads: x over (rest position, j) with j
// fastest, y over groups of R-output chunks of the mode (chunk mc =
// blockIdx.y + k gridDim.y), so the matrix entries are uniform across the
// workgroup and come through the scalar cache.
template <typename TIn, typename TAcc, typename TOut, int R>
__global__ __launch_bounds__(256) void mode_pt_kernel(const TIn* __restrict__ in, int64_t in_ld, TOut* __restrict__ out,
                                                      int64_t out_ld, const TAcc* __restrict__ matT,
                                                      const float* __restrict__ scale, int n0, int n1, int n2,
                                                      int mode, int m, int nv, int64_t nthreads) {
  constexpr int U = 4;   // input values in flight per thread
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nthreads) return;
  const int j = (int)(id % nv);
  const int64_t r = id / nv;
  // the two indices other than `mode`, the first of them fastest
  const int nin[3] = {n0, n1, n2};
  const int da = mode == 0 ? n1 : n0;
  const int ia = (int)(r % da), ib = (int)(r / da);
  int oi[3];
  oi[mode] = 0;
  oi[mode == 0 ? 1 : 0] = ia;
  oi[mode == 2 ? 1 : 2] = ib;
  int no[3] = {n0, n1, n2};
  no[mode] = m;
  const int64_t pin = oi[0] + (int64_t)n0 * (oi[1] + (int64_t)n1 * oi[2]);
  const int64_t pout = oi[0] + (int64_t)no[0] * (oi[1] + (int64_t)no[1] * oi[2]);
  const int64_t sin = mode == 0 ? 1 : (mode == 1 ? (int64_t)n0 : (int64_t)n0 * n1);
  const int64_t sout = mode == 0 ? 1 : (mode == 1 ? (int64_t)no[0] : (int64_t)no[0] * no[1]);
  const int nk = nin[mode];
  const TIn* src = in + pin * in_ld + j;
  const int64_t step = sin * in_ld;
  for (int mc = blockIdx.y; mc * R < m; mc += gridDim.y) {
    const int m0 = mc * R;
    const int rows = m - m0 < R ? m - m0 : R;
    TAcc acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = (TAcc)0;
    // U input values in flight per thread, in full chunks and in the last,
    // partial one alike (there only the chunk's rows are read and summed)
    auto sweep = [&](auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      int c = 0;
      for (; c + U <= nk; c += U) {
        TAcc x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = (TAcc)src[(int64_t)(c + u) * step];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const TAcc* a = matT + (int64_t)(c + u) * m + m0;
#pragma unroll
          for (int q = 0; q < R; ++q)
            if (FULL || q < rows) acc[q] += a[q] * x[u];
        }
      }
      for (; c < nk; ++c) {
        const TAcc x = (TAcc)src[(int64_t)c * step];
        const TAcc* a = matT + (int64_t)c * m + m0;
#pragma unroll
        for (int q = 0; q < R; ++q)
          if (FULL || q < rows) acc[q] += a[q] * x;
      }
    };
    if (rows == R) sweep(std::true_type{});
    else sweep(std::false_type{});
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (q < rows) {
        const int64_t po = pout + (int64_t)(m0 + q) * sout;
        TAcc v = acc[q];
        if (scale) v *= (TAcc)scale[po];
        out[po * out_ld + j] = (TOut)v;
      }
    }
  }
}

// R outputs per thread and pass over the input fiber: 33 for modes longer than
// 32, so that a mode of 66 (the 64^3 cube at p = 2) takes two passes instead
// of five.  Every pass re-reads the fiber, and at that size the re-reads
// come from HBM: 4.8 times the input bytes with R = 16.  Modes of 17 to 32
// keep R = 16: two passes, the first one full, where 33 would make one pass
// with up to half of its accumulators idle.
template <typename TIn, typename TAcc, typename TOut, int R>
static hipError_t launch_mode_pt_r(const ModeArgs& a, hipStream_t s) {
  const int nk = a.n_in[a.mode];
  const int64_t nrest = (int64_t)a.n_in[0] * a.n_in[1] * a.n_in[2] / nk;
  const int64_t nthreads = nrest * a.nv;
  if (nthreads == 0 || a.m == 0) return hipSuccess;
  if (!a.matT) return hipErrorInvalidValue;
  const int chunks = (a.m + R - 1) / R;
  // enough workgroups for small tensors: spread the output chunks over y
  const int gy = (int)std::min<int64_t>(chunks, std::max<int64_t>(1, (65536 + nthreads - 1) / nthreads));
  const dim3 grid((unsigned)((nthreads + 255) / 256), (unsigned)gy);
  hipLaunchKernelGGL((mode_pt_kernel<TIn, TAcc, TOut, R>), grid, dim3(256), 0, s, (const TIn*)a.in, a.in_ld,
                     (TOut*)a.out, a.out_ld, (const TAcc*)a.matT, a.out_scale, a.n_in[0], a.n_in[1], a.n_in[2],
                     a.mode, a.m, a.nv, nthreads);
  return hipGetLastError();
}

template <typename TIn, typename TAcc, typename TOut>
static hipError_t launch_mode_pt(const ModeArgs& a, hipStream_t s) {
  return a.m > 32 ? launch_mode_pt_r<TIn, TAcc, TOut, 33>(a, s) : launch_mode_pt_r<TIn, TAcc, TOut, 16>(a, s);
}

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
  if (a.in_layout == LAYOUT_PT && a.out_layout == LAYOUT_PT) return launch_mode_pt<TIn, TAcc, TOut>(a, s);
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

// Layout changes between the column-major API blocks (element (i, j) at
// i + j ld) and the point-major operator blocks (at i ld + j), through LDS
// tiles of 64 points x 64 vectors so that both sides are read and written in
// memory order.  kPad keeps the transposed LDS reads free of bank conflicts.
constexpr int kTP = 64;
constexpr int kPad = 1;

// point-major TIn (ld_in) -> column-major TOut (ld_out), divided by div[i] if given
template <typename TIn, typename TOut>
__global__ __launch_bounds__(256) void pt_to_col_kernel(const TIn* __restrict__ in, int64_t ld_in,
                                                        TOut* __restrict__ out, int64_t ld_out, int64_t npts, int nv,
                                                        const double* __restrict__ div) {
  __shared__ double t[kTP][kTP + kPad];
  const int64_t p0 = (int64_t)blockIdx.x * kTP;
  const int j0 = blockIdx.y * kTP;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int pp = ty; pp < kTP; pp += 4) {          // read point rows: lanes over vectors
    const int64_t p = p0 + pp;
    const int j = j0 + tx;
    if (p < npts && j < nv) t[pp][tx] = (double)in[p * ld_in + j];
  }
  __syncthreads();
  for (int jj = ty; jj < kTP; jj += 4) {          // write columns: lanes over points
    const int64_t p = p0 + tx;
    const int j = j0 + jj;
    if (p < npts && j < nv) {
      const double v = t[tx][jj];
      out[p + (int64_t)j * ld_out] = (TOut)(div ? v / div[p] : v);
    }
  }
}

// column-major double (ld_in) -> point-major double (ld_out)
__global__ __launch_bounds__(256) void col_to_pt_kernel(const double* __restrict__ in, int64_t ld_in,
                                                        double* __restrict__ out, int64_t ld_out, int64_t npts,
                                                        int nv) {
  __shared__ double t[kTP][kTP + kPad];
  const int64_t p0 = (int64_t)blockIdx.x * kTP;
  const int j0 = blockIdx.y * kTP;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int jj = ty; jj < kTP; jj += 4) {          // read columns: lanes over points
    const int64_t p = p0 + tx;
    const int j = j0 + jj;
    if (p < npts && j < nv) t[jj][tx] = in[p + (int64_t)j * ld_in];
  }
  __syncthreads();
  for (int pp = ty; pp < kTP; pp += 4) {          // write point rows: lanes over vectors
    const int64_t p = p0 + pp;
    const int j = j0 + tx;
    if (p < npts && j < nv) out[p * ld_out + j] = t[tx][pp];
  }
}

static dim3 tile_grid(int64_t npts, int nv) {
  return dim3((unsigned)((npts + kTP - 1) / kTP), (unsigned)((nv + kTP - 1) / kTP));
}

hipError_t cast_pt32_to_col64(const float* in, int64_t ld_in, double* out, int64_t ld_out, int64_t npts, int nv,
                              const double* div, hipStream_t s) {
  if (npts * nv == 0) return hipSuccess;
  hipLaunchKernelGGL((pt_to_col_kernel<float, double>), tile_grid(npts, nv), dim3(256), 0, s, in, ld_in, out, ld_out,
                     npts, nv, div);
  return hipGetLastError();
}

hipError_t pt64_to_col64(const double* in, int64_t ld_in, double* out, int64_t ld_out, int64_t npts, int nv,
                         hipStream_t s) {
  if (npts * nv == 0) return hipSuccess;
  hipLaunchKernelGGL((pt_to_col_kernel<double, double>), tile_grid(npts, nv), dim3(256), 0, s, in, ld_in, out,
                     ld_out, npts, nv, nullptr);
  return hipGetLastError();
}

hipError_t col64_to_pt64(const double* in, int64_t ld_in, double* out, int64_t ld_out, int64_t npts, int nv,
                         hipStream_t s) {
  if (npts * nv == 0) return hipSuccess;
  hipLaunchKernelGGL(col_to_pt_kernel, tile_grid(npts, nv), dim3(256), 0, s, in, ld_in, out, ld_out, npts, nv);
  return hipGetLastError();
}

}  // namespace ka
