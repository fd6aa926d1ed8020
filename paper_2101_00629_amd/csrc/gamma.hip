// Fused covariance-kernel product Z = out_scale * diag(rs) * Gamma * Y with
// Gamma[r][c] = exp2(-s(xr_r - xc_c)) evaluated on the fly and never stored.
//
// This is the quadratic-cost step of both matrix-free operators: the Gamma
// product of the Galerkin nine-step algorithm (paper Sec. 3.1) and step 3 of
// Algorithm 1 (paper Sec. 3.2).  Coordinates are prescaled so that the kernel
// is a bare exp2:
//   Gaussian     s = |d|_2^2  with coordinates scaled by sqrt(log2 e) / ell,
//   exponential  s = |d|_1    with coordinates scaled by log2 e / ell.
//
// Work decomposition (gfx950, wave64):
//   * a workgroup of 4 waves owns 4*16*RB consecutive rows; each wave owns RB
//     16-row sub-blocks whose coordinates live in registers;
//   * columns stream through LDS in tiles of CT points (coordinates + the
//     matching rows of Y), double buffered, one barrier per tile;
//   * per MFMA step every lane evaluates the kernel for its (row, column)
//     slots straight into the A-operand register(s) of the matrix core; the
//     B operand is the matching slice of Y; accumulators stay in AGPRs;
//   * FP32 path: v_mfma_f32_16x16x4_f32, one pair per lane per step, B/16
//     MFMAs per pair (one per 16 columns of Y);
//   * BF16x3 path: v_mfma_f32_16x16x32_bf16, eight pairs per lane per step,
//     Gamma and Y split into hi + lo BF16 parts, products hi*hi + hi*lo +
//     lo*hi accumulated in FP32;
//   * the column range is split over gridDim.y (split-K) when there are too
//     few row blocks to fill the chip; partial results go to a scratch array
//     and are summed in a fixed split order, so results depend only on the
//     shape, never on what else runs on the device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ka_internal.hpp"

namespace ka {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;
constexpr int kXcds = 8;        // MI355X: workgroups are dealt to the 8 XCDs round-robin by id
constexpr int kCT = 64;         // columns per LDS tile
// MFMA accumulators are flushed into running totals every 2 tiles (128
// columns, 32 chained MFMAs per FP32 accumulator): FP64 totals in the FP32
// path, FP32 totals in the BF16x3 path.  The FP32 chain length is
// what sets the arithmetic noise of the product: measured on the 287,496-point
// Gaussian operator, 8-tile chains gave 1.8e-6 relative error on the smallest
// of 200 eigenvalues (1.4% of the largest), 2-tile chains 3.8e-7, at the same
// speed within 1%.
constexpr int kFlushTiles = 2;
constexpr double kL2FitBytes = 3.0 * (1 << 20);   // column data per split that an XCD's L2 keeps


// (row block, split) of this workgroup.  Grouped grid (xcd_splits > 0): a 1-D
// grid of row_blocks * xcd_splits workgroups; workgroup id L runs on XCD
// L % 8, and the XCD's own sequence L / 8 walks split by split (all row
// blocks of a split back to back), splits x, x + 8, ... on XCD x.  Returns
// false for padding workgroups (split beyond the real split count).
__device__ __forceinline__ bool gamma_item(const GammaLaunch& a, int64_t& rblk, int& split) {
  if (a.xcd_splits == 0) {
    rblk = blockIdx.x;
    split = blockIdx.y;
    return true;
  }
  const int64_t L = blockIdx.x;
  const int x = (int)(L % kXcds);
  const int64_t j = L / kXcds;
  rblk = j % a.row_blocks;
  split = x + kXcds * (int)(j / a.row_blocks);
  return split < a.nsplit;
}

template <int KERNEL>
__device__ __forceinline__ float pair_exponent(float dx, float dy, float dz) {
  if constexpr (KERNEL == KA_GAUSSIAN) {
    float s = dx * dx;
    s = __builtin_fmaf(dy, dy, s);
    return __builtin_fmaf(dz, dz, s);
  } else {
    return (__builtin_fabsf(dx) + __builtin_fabsf(dy)) + __builtin_fabsf(dz);
  }
}

__device__ __forceinline__ float load_coord(const float* p, int64_t i, int stride, int k, float scale) {
  return p[i * stride + k] * scale;
}

// ---------------------------------------------------------------------------
// FP32 path
// ---------------------------------------------------------------------------
// LDS row stride of Y in the FP32 path (spreads the 16-lane groups over banks)
template <int B>
constexpr int y_stride() { return (B == 16) ? 16 : B + 16; }

// Centred Gram form of the Gaussian exponent (FP32 path).  With c the centre
// of the bounding box of a workgroup's rows, xt = x - c and yt = y - c (scaled
// coordinates),
//     2^-|x - y|^2 = 2^-|xt|^2 * 2^((2 yt) . xt - |yt|^2),
// so the exponents of 16 x 16 pairs, less the row term, are one
// v_mfma_f32_16x16x4_f32: A holds (2 yt, -|yt|^2) of 16 columns and B holds
// (xt, 1) of 16 rows; the row factor 2^-|xt|^2 multiplies the finished row of
// the product.  Lane l of the result holds row l % 16 against four columns,
// which is where the kernel product's A operand expects Gamma when column
// 4 * (m % 4) + m / 4 of the group is put in A row m: result entry r of lane l
// is then column 4 r + l / 16, the column of k-slot l / 16 in product step
// 4 r.  This replaces three differences and three multiply-adds per pair by
// 1/64 of an MFMA.  Rounding: the terms are of size R^2 (R the half-diagonal
// of the rows' box) where the difference form's are of size |x - y|^2, so the
// form is taken only for boxes with R^2 <= kGramR2 in scaled units (the
// exponent is then off by a few units of 2^-24 R^2 at most, Gamma by ln 2
// times that relative, and the factored terms stay below 2^(R^2)); wider row
// blocks keep the difference form.  Row blocks of tensor-grid points in their
// natural order qualify at the workload sizes: R^2 = 9.0 on the 66^3 cube at
// ell = 0.2 (18.0 for the blocks that straddle two z-layers), at most 11.5 on
// the quarter annulus r in [1, 2] at ell = 0.5.  The cut takes in the
// straddling blocks on purpose: workgroups of one launch that run the two
// forms at different speeds drift apart in their column streams and stop
// sharing the XCD's L2 (measured on the 66^3 launch with a cut of 16: 5x the
// HBM fetch, 29.7 GB against 5.9 GB per launch).
constexpr float kGramR2 = 20.f;

// Bounding box of a wave's rows (lanes l and l + 16 hold the same rows) into
// the wave's entry of s_box: lo in [0..2], hi in [4..6].
template <int RB>
__device__ __forceinline__ void gram_box_put(const float* rx, const float* ry, const float* rz, int lane, int wave,
                                             float (*s_box)[8]) {
  float lo[3] = {rx[0], ry[0], rz[0]}, hi[3] = {rx[0], ry[0], rz[0]};
#pragma unroll
  for (int rb = 1; rb < RB; ++rb) {
    lo[0] = fminf(lo[0], rx[rb]); hi[0] = fmaxf(hi[0], rx[rb]);
    lo[1] = fminf(lo[1], ry[rb]); hi[1] = fmaxf(hi[1], ry[rb]);
    lo[2] = fminf(lo[2], rz[rb]); hi[2] = fmaxf(hi[2], rz[rb]);
  }
#pragma unroll
  for (int o = 1; o < 16; o <<= 1)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], o));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], o));
    }
  if (lane < 3) {
    s_box[wave][lane] = lane == 0 ? lo[0] : (lane == 1 ? lo[1] : lo[2]);
    s_box[wave][4 + lane] = lane == 0 ? hi[0] : (lane == 1 ? hi[1] : hi[2]);
  }
}

// After gram_box_put on every wave: a barrier, then the centre of the
// workgroup's box and whether the Gram form applies (uniform over the
// workgroup).  The barrier also orders this read before any later rewrite of
// s_box: every wave passes at least one more barrier before its next item.
__device__ __forceinline__ bool gram_box_take(float (*s_box)[8], float& cx, float& cy, float& cz) {
  __syncthreads();
  float lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = fminf(fminf(s_box[0][k], s_box[1][k]), fminf(s_box[2][k], s_box[3][k]));
    hi[k] = fmaxf(fmaxf(s_box[0][4 + k], s_box[1][4 + k]), fmaxf(s_box[2][4 + k], s_box[3][4 + k]));
  }
  cx = 0.5f * (lo[0] + hi[0]);
  cy = 0.5f * (lo[1] + hi[1]);
  cz = 0.5f * (lo[2] + hi[2]);
  const float ex = 0.5f * (hi[0] - lo[0]), ey = 0.5f * (hi[1] - lo[1]), ez = 0.5f * (hi[2] - lo[2]);
  return __builtin_amdgcn_readfirstlane((int)(ex * ex + ey * ey + ez * ez <= kGramR2)) != 0;
}

// A-operand data of one column in the Gram form: (2 yt, -|yt|^2) from the raw
// coordinates.
__device__ __forceinline__ float4 gram_column(float4 raw, float scale, float cx, float cy, float cz) {
  const float tx = raw.x * scale - cx, ty = raw.y * scale - cy, tz = raw.z * scale - cz;
  return make_float4(2.f * tx, 2.f * ty, 2.f * tz, -__builtin_fmaf(tz, tz, __builtin_fmaf(ty, ty, tx * tx)));
}

// The row factor 2^-|xt|^2 of the Gram form.
__device__ __forceinline__ double gram_row_factor(const GammaLaunch& a, int64_t row, float cx, float cy, float cz) {
  const float tx = load_coord(a.xr, row, a.xr_stride, 0, a.coord_scale) - cx;
  const float ty = load_coord(a.xr, row, a.xr_stride, 1, a.coord_scale) - cy;
  const float tz = load_coord(a.xr, row, a.xr_stride, 2, a.coord_scale) - cz;
  return exp2(-(double)__builtin_fmaf(tz, tz, __builtin_fmaf(ty, ty, tx * tx)));
}

// Row box of a work item and whether the centred Gram form applies to it
// (Gaussian kernel only); contains a workgroup barrier.
template <int RB>
__device__ __forceinline__ bool gram_rows(const GammaLaunch& a, int64_t rblk, float (*s_box)[8], float& cx,
                                          float& cy, float& cz) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = rblk * (4 * 16 * RB) + wave * 16 * RB;
  float rx[RB], ry[RB], rz[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    int64_t r = row0 + 16 * rb + (lane & 15);
    if (r >= a.nr) r = a.nr - 1;
    rx[rb] = load_coord(a.xr, r, a.xr_stride, 0, a.coord_scale);
    ry[rb] = load_coord(a.xr, r, a.xr_stride, 1, a.coord_scale);
    rz[rb] = load_coord(a.xr, r, a.xr_stride, 2, a.coord_scale);
  }
  gram_box_put<RB>(rx, ry, rz, lane, wave, s_box);
  return gram_box_take(s_box, cx, cy, cz);
}

// One work item: rows [rblk * ROWS, +ROWS) against the column range of split
// `split` of one kernel product.  LDS buffers are provided by the caller.
template <int KERNEL, int B, int RB>
__device__ __forceinline__ void gamma_f32_tile(const GammaLaunch& a, int64_t rblk, int split,
                                               float4 (*s_x)[kCT], float (*s_y)[kCT * y_stride<B>()]) {
  constexpr int NT = B / 16;
  constexpr int YS = y_stride<B>();
  constexpr int ROWS = 4 * 16 * RB;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = rblk * ROWS + wave * 16 * RB;
  const int64_t c_begin = (int64_t)split * a.cols_per_split;
  const int64_t c_end = (c_begin + a.cols_per_split < a.nc) ? c_begin + a.cols_per_split : a.nc;

  float rx[RB], ry[RB], rz[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    int64_t r = row0 + 16 * rb + (lane & 15);
    if (r >= a.nr) r = a.nr - 1;
    rx[rb] = load_coord(a.xr, r, a.xr_stride, 0, a.coord_scale);
    ry[rb] = load_coord(a.xr, r, a.xr_stride, 1, a.coord_scale);
    rz[rb] = load_coord(a.xr, r, a.xr_stride, 2, a.coord_scale);
  }

  f4v acc[RB][NT];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[rb][t] = (f4v){0.f, 0.f, 0.f, 0.f};
  // Two-level summation: MFMA chains of at most kFlushTiles tiles are added
  // into FP64 running totals, so the FP32 rounding error grows only with the
  // chain length, never with the column count.
  d4v tot[RB][NT];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int t = 0; t < NT; ++t) tot[rb][t] = (d4v){0.0, 0.0, 0.0, 0.0};
  auto flush = [&]() {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        tot[rb][t] += __builtin_convertvector(acc[rb][t], d4v);
        acc[rb][t] = (f4v){0.f, 0.f, 0.f, 0.f};
      }
  };

  // per-thread staging registers for one tile
  constexpr int YV = kCT * B / 4 / kThreads;   // float4 of Y per thread per tile
  float4 ybuf[YV];
  float4 xbuf;

  // A tile's addresses are a base common to the workgroup plus a 32-bit
  // offset per thread that does not change from tile to tile, and the range
  // test compares the tile row with the rows left, so no 64-bit address
  // arithmetic or compare runs per load.
  auto fetch = [&](int64_t ct) {
    const float* yt = a.Y + ct * B;
    const int64_t left = c_end - ct;
    const int rem = left < kCT ? (int)left : kCT;   // rows of this tile in range
#pragma unroll
    for (int v = 0; v < YV; ++v) {
      const int e = (threadIdx.x + v * kThreads) * 4;   // element in tile (b fastest)
      const int row = e / B;
      ybuf[v] = row < rem ? *reinterpret_cast<const float4*>(yt + (row * B + e % B))
                          : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // raw coordinates: the scale is applied in stash(), after the tile's work,
    // so no wait for these loads (which would also wait for Y) lands here
    if (threadIdx.x < kCT) {
      const float* xt = a.xc + ct * a.xc_stride;
      const int o = (int)threadIdx.x * a.xc_stride;
      if ((int)threadIdx.x < rem)
        xbuf = make_float4(xt[o], xt[o + 1], xt[o + 2], 0.f);
      else
        xbuf = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int v = 0; v < YV; ++v) {
      const int e = (threadIdx.x + v * kThreads) * 4;
      float* dst = &s_y[buf][(e / B) * YS + (e % B)];
      dst[0] = ybuf[v].x; dst[1] = ybuf[v].y; dst[2] = ybuf[v].z; dst[3] = ybuf[v].w;
    }
    if (threadIdx.x < kCT)
      s_x[buf][threadIdx.x] = make_float4(xbuf.x * a.coord_scale, xbuf.y * a.coord_scale, xbuf.z * a.coord_scale, 0.f);
  };

  int buf = 0;
  fetch(c_begin);
  stash(0);
  __syncthreads();
  // Tiles go in groups of kFlushTiles with an unconditional flush after each
  // group, so the MFMA accumulators enter every group at zero and are never
  // carried around the loop.  The next tile is always fetched: beyond c_end
  // it is zero-filled (Y = 0), so a padding tile in the last group adds
  // exactly zero.
  for (int64_t cg = c_begin; cg < c_end; cg += kFlushTiles * kCT) {
#pragma unroll
  for (int f = 0; f < kFlushTiles; ++f) {
    const int64_t ct = cg + f * kCT;
    fetch(ct + kCT);
    // Fully unrolled: with a rolled loop the register allocator rotates the
    // accumulators through AGPR copies every step (measured at b = 64: 40
    // extra VALU instructions per 16 MFMAs).  The LDS operands of step k + 1
    // are read before step k is computed, and a scheduling barrier keeps the
    // compiler from sinking those reads back to their use, so every LDS read
    // has one whole step of work to complete in (measured: +4-5% at b = 16).
    float4 pc = s_x[buf][lane >> 4];
    float yc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) yc[t] = s_y[buf][(lane >> 4) * YS + 16 * t + (lane & 15)];
#pragma unroll
    for (int k = 0; k < kCT; k += 4) {
      const float4 p = pc;
      float yv[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) yv[t] = yc[t];
      if (k + 4 < kCT) {
        const int cn = k + 4 + (lane >> 4);
        pc = s_x[buf][cn];
#pragma unroll
        for (int t = 0; t < NT; ++t) yc[t] = s_y[buf][cn * YS + 16 * t + (lane & 15)];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const float g = __builtin_amdgcn_exp2f(-pair_exponent<KERNEL>(rx[rb] - p.x, ry[rb] - p.y, rz[rb] - p.z));
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[rb][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(g, yv[t], acc[rb][t], 0, 0, 0);
      }
    }
    stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
    flush();
  }

  float* out = a.nsplit > 1 ? a.partial + (size_t)split * a.nr * B : a.Z;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + 16 * rb + 4 * (lane >> 4) + r;
      if (row < a.nr) {
        const float sc = a.out_scale * (a.rs ? a.rs[row] : 1.0f);
#pragma unroll
        for (int t = 0; t < NT; ++t) out[row * B + 16 * t + (lane & 15)] = (float)((double)sc * tot[rb][t][r]);
      }
    }
  }
}

// The FP32 tile in the centred Gram form (Gaussian kernel, centre c of the
// rows' box): per group of 16 columns and row sub-block one Gram MFMA gives
// the exponents, computed one group ahead of the product steps that use them.
template <int B, int RB>
__device__ __forceinline__ void gamma_f32_gram_tile(const GammaLaunch& a, int64_t rblk, int split,
                                                    float4 (*s_x)[kCT], float (*s_y)[kCT * y_stride<B>()],
                                                    float cx, float cy, float cz) {
  constexpr int NT = B / 16;
  constexpr int YS = y_stride<B>();
  constexpr int ROWS = 4 * 16 * RB;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = rblk * ROWS + wave * 16 * RB;
  const int64_t c_begin = (int64_t)split * a.cols_per_split;
  const int64_t c_end = (c_begin + a.cols_per_split < a.nc) ? c_begin + a.cols_per_split : a.nc;

  // B operand (xt, 1) of each row sub-block
  float bx[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    int64_t r = row0 + 16 * rb + (lane & 15);
    if (r >= a.nr) r = a.nr - 1;
    const int q = lane >> 4;
    const float v = q < 3 ? load_coord(a.xr, r, a.xr_stride, q, a.coord_scale) : 0.f;
    bx[rb] = q == 0 ? v - cx : (q == 1 ? v - cy : (q == 2 ? v - cz : 1.f));
  }
  const f4v zero4 = {0.f, 0.f, 0.f, 0.f};

  f4v acc[RB][NT];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[rb][t] = (f4v){0.f, 0.f, 0.f, 0.f};
  d4v tot[RB][NT];   // FP64 running totals, as in the difference form
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int t = 0; t < NT; ++t) tot[rb][t] = (d4v){0.0, 0.0, 0.0, 0.0};
  auto flush = [&]() {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        tot[rb][t] += __builtin_convertvector(acc[rb][t], d4v);
        acc[rb][t] = (f4v){0.f, 0.f, 0.f, 0.f};
      }
  };

  constexpr int YV = kCT * B / 4 / kThreads;
  float4 ybuf[YV];
  float4 xbuf;
  auto fetch = [&](int64_t ct) {
    const float* yt = a.Y + ct * B;
    const int64_t left = c_end - ct;
    const int rem = left < kCT ? (int)left : kCT;
#pragma unroll
    for (int v = 0; v < YV; ++v) {
      const int e = (threadIdx.x + v * kThreads) * 4;
      const int row = e / B;
      ybuf[v] = row < rem ? *reinterpret_cast<const float4*>(yt + (row * B + e % B))
                          : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (threadIdx.x < kCT) {
      const float* xt = a.xc + ct * a.xc_stride;
      const int o = (int)threadIdx.x * a.xc_stride;
      if ((int)threadIdx.x < rem)
        xbuf = make_float4(xt[o], xt[o + 1], xt[o + 2], 0.f);
      else
        xbuf = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int v = 0; v < YV; ++v) {
      const int e = (threadIdx.x + v * kThreads) * 4;
      float* dst = &s_y[buf][(e / B) * YS + (e % B)];
      dst[0] = ybuf[v].x; dst[1] = ybuf[v].y; dst[2] = ybuf[v].z; dst[3] = ybuf[v].w;
    }
    if (threadIdx.x < kCT) s_x[buf][threadIdx.x] = gram_column(xbuf, a.coord_scale, cx, cy, cz);
  };

  int buf = 0;
  fetch(c_begin);
  stash(0);
  __syncthreads();
  // A operand of the Gram MFMA: component l / 16 of column 4 (m % 4) + m / 4
  // of the group, m = l % 16
  const int aoff = 4 * (4 * (lane & 3) + ((lane >> 2) & 3)) + (lane >> 4);
  for (int64_t cg = c_begin; cg < c_end; cg += kFlushTiles * kCT) {
#pragma unroll
    for (int f = 0; f < kFlushTiles; ++f) {
      const int64_t ct = cg + f * kCT;
      fetch(ct + kCT);
      // LDS operands one step ahead, held there by a scheduling barrier, as
      // in the difference form
      float yc[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) yc[t] = s_y[buf][(lane >> 4) * YS + 16 * t + (lane & 15)];
      const float* sxf = reinterpret_cast<const float*>(&s_x[buf][0]);
      f4v dcur[RB], dnext[RB];
      {
        const float ad = sxf[aoff];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) dcur[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ad, bx[rb], zero4, 0, 0, 0);
      }
#pragma unroll
      for (int k = 0; k < kCT; k += 4) {
        float yv[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) yv[t] = yc[t];
        float adn = 0.f;
        if (k + 4 < kCT) {
          const int cn = k + 4 + (lane >> 4);
#pragma unroll
          for (int t = 0; t < NT; ++t) yc[t] = s_y[buf][cn * YS + 16 * t + (lane & 15)];
        }
        if (k % 16 == 0 && k + 16 < kCT) adn = sxf[4 * (k + 16) + aoff];
        __builtin_amdgcn_sched_barrier(0);
        if (k % 16 == 0 && k + 16 < kCT) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            dnext[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(adn, bx[rb], zero4, 0, 0, 0);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const float g = __builtin_amdgcn_exp2f(dcur[rb][(k / 4) % 4]);
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc[rb][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(g, yv[t], acc[rb][t], 0, 0, 0);
        }
        if (k % 16 == 12 && k + 4 < kCT) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) dcur[rb] = dnext[rb];
        }
      }
      stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
    flush();
  }

  float* out = a.nsplit > 1 ? a.partial + (size_t)split * a.nr * B : a.Z;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + 16 * rb + 4 * (lane >> 4) + r;
      if (row < a.nr) {
        const float sc = a.out_scale * (a.rs ? a.rs[row] : 1.0f);
        const double f = sc * gram_row_factor(a, row, cx, cy, cz);
#pragma unroll
        for (int t = 0; t < NT; ++t) out[row * B + 16 * t + (lane & 15)] = (float)(f * tot[rb][t][r]);
      }
    }
  }
}

// One FP32 work item: the Gram form where it applies, else the difference
// form.
template <int KERNEL, int B, int RB>
__device__ __forceinline__ void gamma_f32_item(const GammaLaunch& a, int64_t rblk, int split, float4 (*s_x)[kCT],
                                               float (*s_y)[kCT * y_stride<B>()], float (*s_box)[8]) {
  if constexpr (KERNEL == KA_GAUSSIAN) {
    float cx, cy, cz;
    if (gram_rows<RB>(a, rblk, s_box, cx, cy, cz)) {
      gamma_f32_gram_tile<B, RB>(a, rblk, split, s_x, s_y, cx, cy, cz);
      return;
    }
  }
  gamma_f32_tile<KERNEL, B, RB>(a, rblk, split, s_x, s_y);
}

// Occupancy target of the FP32 path (waves per SIMD).  FP32 MFMA and VALU
// work do not overlap on gfx950, so the kernel is issue bound; the target
// trades latency hiding against registers for scheduling.  Measured best on
// the workload shapes: 4 at b = 16, 3 at b = 32, 2 at b = 64.
template <int B>
constexpr int f32_waves() { return B == 16 ? 4 : (B == 32 ? 3 : 2); }

template <int KERNEL, int B, int RB>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(f32_waves<B>(), f32_waves<B>())))
void gamma_f32_kernel(GammaLaunch a) {
  __shared__ float4 s_x[2][kCT];
  __shared__ float s_y[2][kCT * y_stride<B>()];
  __shared__ float s_box[4][8];
  int64_t rblk;
  int split;
  if (!gamma_item(a, rblk, split)) return;
  gamma_f32_item<KERNEL, B, RB>(a, rblk, split, s_x, s_y, s_box);
}

// ---------------------------------------------------------------------------
// split hi/lo BF16 path
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pack_bf16x2(float lo_elem, float hi_elem) {
  bf2v h = {(__bf16)lo_elem, (__bf16)hi_elem};
  return __builtin_bit_cast(uint32_t, h);
}

// Split two FP32 values into packed BF16 hi and lo words (round to nearest
// even for both; x - hi is exact in FP32).
__device__ __forceinline__ void split2(float x0, float x1, uint32_t& hi, uint32_t& lo) {
  hi = pack_bf16x2(x0, x1);
  // low half of hi moved to the top, zeros below (one v_perm_b32; written as
  // a shift the compiler re-converts x0 instead)
  const float h0 = __builtin_bit_cast(float, __builtin_amdgcn_perm(0u, hi, 0x01000c0cu));
  const float h1 = __builtin_bit_cast(float, hi & 0xffff0000u);
  lo = pack_bf16x2(x0 - h0, x1 - h1);
}

constexpr int kKS = kCT / 32;   // BF16 MFMA k-steps per tile

// Y split once per product for the BF16x3 path, straight into the order the
// kernel's LDS buffers hold the MFMA B operands.  Entry r of 64-column tile T
// (r = (ks * NT + t) * 64 + lane, lane = 16 * grp + n) is the fragment of Y
// column j = 16 t + n over the 8 tile columns 32 ks + 8 grp + u, u = 0..7,
// as 8 BF16 values; hi parts at ys[2 E T + r], lo parts at ys[2 E T + E + r]
// (E entries per tile and part).  Columns past nc are zero.
template <int B>
__device__ __forceinline__ void split_y_entry(const float* __restrict__ Y, int64_t nc, uint4* __restrict__ ys,
                                              int64_t e) {
  constexpr int NT = B / 16;
  constexpr int E = kKS * NT * 64;
  const int64_t T = e / E;
  const int r = (int)(e - T * E);
  const int lane = r & 63, t = (r >> 6) % NT, ks = r / (64 * NT);
  const int j = 16 * t + (lane & 15);
  const int64_t c0 = kCT * T + 32 * ks + 8 * (lane >> 4);
  float y[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) y[u] = (c0 + u < nc) ? Y[(c0 + u) * B + j] : 0.f;
  uint4 h, l;
  split2(y[0], y[1], h.x, l.x);
  split2(y[2], y[3], h.y, l.y);
  split2(y[4], y[5], h.z, l.z);
  split2(y[6], y[7], h.w, l.w);
  ys[2 * E * T + r] = h;
  ys[2 * E * T + E + r] = l;
}

template <int B>
constexpr int64_t split_entries(int64_t nc) { return (nc + kCT - 1) / kCT * (kKS * (B / 16) * 64); }

template <int B>
__global__ __launch_bounds__(256) void gamma_split_kernel(const float* __restrict__ Y, int64_t nc,
                                                          uint4* __restrict__ ys) {
  const int64_t n = split_entries<B>(nc);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    split_y_entry<B>(Y, nc, ys, e);
}

// B-operand fragments in LDS: [k-step][t][lane] -> 4 dwords (8 bf16)
template <int KERNEL, int B, int RB>
__device__ __forceinline__ void gamma_bf16x3_tile(const GammaLaunch& a, int64_t rblk, int split,
                                                  float4 (*s_x)[kCT], uint4 (*s_yh)[kKS * (B / 16) * 64],
                                                  uint4 (*s_yl)[kKS * (B / 16) * 64]) {
  constexpr int NT = B / 16;
  constexpr int KS = kKS;
  constexpr int ROWS = 4 * 16 * RB;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = rblk * ROWS + wave * 16 * RB;
  const int64_t c_begin = (int64_t)split * a.cols_per_split;
  const int64_t c_end = (c_begin + a.cols_per_split < a.nc) ? c_begin + a.cols_per_split : a.nc;

  float rx[RB], ry[RB], rz[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    int64_t r = row0 + 16 * rb + (lane & 15);
    if (r >= a.nr) r = a.nr - 1;
    rx[rb] = load_coord(a.xr, r, a.xr_stride, 0, a.coord_scale);
    ry[rb] = load_coord(a.xr, r, a.xr_stride, 1, a.coord_scale);
    rz[rb] = load_coord(a.xr, r, a.xr_stride, 2, a.coord_scale);
  }

  f4v acc[RB][NT];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[rb][t] = (f4v){0.f, 0.f, 0.f, 0.f};
  // Two-level summation as in the FP32 path, but with FP32 running totals:
  // the BF16 representation of Gamma (about 2^-17 relative) dominates the
  // error here, and the 32 registers FP64 totals would take decide the
  // occupancy (measured at b = 64: 3 waves per SIMD instead of 2, +10%).
  f4v tot[RB][NT];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int t = 0; t < NT; ++t) tot[rb][t] = (f4v){0.f, 0.f, 0.f, 0.f};
  auto flush = [&]() {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        tot[rb][t] += acc[rb][t];
        acc[rb][t] = (f4v){0.f, 0.f, 0.f, 0.f};
      }
  };

  // staging: the tile's hi and lo B fragments are contiguous in the
  // pre-split Y (gamma_split_y), in the order the LDS buffers hold them.
  constexpr int E = KS * NT * 64;                    // uint4 per tile and part
  constexpr int FPT = (E + kThreads - 1) / kThreads; // per thread (b = 16: threads 0..127 only)
  uint4 hbuf[FPT], lbuf[FPT];
  float4 xbuf;

  auto fetch = [&](int64_t ct) {
    const uint4* src = a.ys + (ct / kCT) * (2 * E);
    const bool in = ct < c_end;   // uniform: tiles past the split end stage zeros
#pragma unroll
    for (int v = 0; v < FPT; ++v) {
      const int e = threadIdx.x + v * kThreads;
      if (e < E) {
        hbuf[v] = in ? src[e] : make_uint4(0u, 0u, 0u, 0u);
        lbuf[v] = in ? src[E + e] : make_uint4(0u, 0u, 0u, 0u);
      }
    }
    // raw coordinates: the scale is applied in stash(), after the tile's work,
    // so no wait for these loads (which would also wait for Y) lands here;
    // a shared base plus a 32-bit offset per thread, as in the FP32 path
    if (threadIdx.x < kCT) {
      const float* xt = a.xc + ct * a.xc_stride;
      const int o = (int)threadIdx.x * a.xc_stride;
      if ((int64_t)threadIdx.x < c_end - ct)
        xbuf = make_float4(xt[o], xt[o + 1], xt[o + 2], 0.f);
      else
        xbuf = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int v = 0; v < FPT; ++v) {
      const int e = threadIdx.x + v * kThreads;
      if (e < E) {
        s_yh[buf][e] = hbuf[v];
        s_yl[buf][e] = lbuf[v];
      }
    }
    if (threadIdx.x < kCT)
      s_x[buf][threadIdx.x] = make_float4(xbuf.x * a.coord_scale, xbuf.y * a.coord_scale, xbuf.z * a.coord_scale, 0.f);
  };

  int buf = 0;
  fetch(c_begin);
  stash(0);
  __syncthreads();
  // Tile groups with an unconditional flush, as in the FP32 path.
  for (int64_t cg = c_begin; cg < c_end; cg += kFlushTiles * kCT) {
#pragma unroll
  for (int f = 0; f < kFlushTiles; ++f) {
    const int64_t ct = cg + f * kCT;
    fetch(ct + kCT);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      float4 p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) p[u] = s_x[buf][ks * 32 + 8 * (lane >> 4) + u];
      bf8v yh[NT], yl[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        yh[t] = __builtin_bit_cast(bf8v, s_yh[buf][(ks * NT + t) * 64 + lane]);
        yl[t] = __builtin_bit_cast(bf8v, s_yl[buf][(ks * NT + t) * 64 + lane]);
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        float g[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          g[u] = __builtin_amdgcn_exp2f(-pair_exponent<KERNEL>(rx[rb] - p[u].x, ry[rb] - p[u].y, rz[rb] - p[u].z));
        uint4 gh, gl;
        split2(g[0], g[1], gh.x, gl.x);
        split2(g[2], g[3], gh.y, gl.y);
        split2(g[4], g[5], gh.z, gl.z);
        split2(g[6], g[7], gh.w, gl.w);
        const bf8v ah = __builtin_bit_cast(bf8v, gh);
        const bf8v al = __builtin_bit_cast(bf8v, gl);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          acc[rb][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, yh[t], acc[rb][t], 0, 0, 0);
          acc[rb][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, yl[t], acc[rb][t], 0, 0, 0);
          acc[rb][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, yh[t], acc[rb][t], 0, 0, 0);
        }
      }
    }
    stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
    flush();
  }

  float* out = a.nsplit > 1 ? a.partial + (size_t)split * a.nr * B : a.Z;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + 16 * rb + 4 * (lane >> 4) + r;
      if (row < a.nr) {
        const float sc = a.out_scale * (a.rs ? a.rs[row] : 1.0f);
#pragma unroll
        for (int t = 0; t < NT; ++t) out[row * B + 16 * t + (lane & 15)] = (float)((double)sc * tot[rb][t][r]);
      }
    }
  }
}

// The BF16x3 tile in the centred Gram form of the FP32 path (Gaussian kernel,
// centre c of the rows' box).  The 8 columns 32 ks + 8 (l / 16) + u of lane
// l's A operand come from two Gram MFMAs, the first over columns
// 32 ks + 8 (m / 4) + m % 4 in A row m (u = 0..3 in result entries 0..3), the
// second over the same columns + 4 (u = 4..7), so the pre-split Y keeps its
// layout.  Per pair this leaves the exp2 and the hi/lo split on the VALU.
template <int B, int RB>
__device__ __forceinline__ void gamma_bf16x3_gram_tile(const GammaLaunch& a, int64_t rblk, int split,
                                                       float4 (*s_x)[kCT], uint4 (*s_yh)[kKS * (B / 16) * 64],
                                                       uint4 (*s_yl)[kKS * (B / 16) * 64], float cx, float cy,
                                                       float cz) {
  constexpr int NT = B / 16;
  constexpr int KS = kKS;
  constexpr int ROWS = 4 * 16 * RB;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = rblk * ROWS + wave * 16 * RB;
  const int64_t c_begin = (int64_t)split * a.cols_per_split;
  const int64_t c_end = (c_begin + a.cols_per_split < a.nc) ? c_begin + a.cols_per_split : a.nc;

  // B operand (xt, 1) of each row sub-block
  float bx[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    int64_t r = row0 + 16 * rb + (lane & 15);
    if (r >= a.nr) r = a.nr - 1;
    const int q = lane >> 4;
    const float v = q < 3 ? load_coord(a.xr, r, a.xr_stride, q, a.coord_scale) : 0.f;
    bx[rb] = q == 0 ? v - cx : (q == 1 ? v - cy : (q == 2 ? v - cz : 1.f));
  }
  const f4v zero4 = {0.f, 0.f, 0.f, 0.f};

  f4v acc[RB][NT];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[rb][t] = (f4v){0.f, 0.f, 0.f, 0.f};
  f4v tot[RB][NT];   // FP32 running totals, as in the difference form
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int t = 0; t < NT; ++t) tot[rb][t] = (f4v){0.f, 0.f, 0.f, 0.f};
  auto flush = [&]() {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        tot[rb][t] += acc[rb][t];
        acc[rb][t] = (f4v){0.f, 0.f, 0.f, 0.f};
      }
  };

  constexpr int E = KS * NT * 64;
  constexpr int FPT = (E + kThreads - 1) / kThreads;
  uint4 hbuf[FPT], lbuf[FPT];
  float4 xbuf;

  auto fetch = [&](int64_t ct) {
    const uint4* src = a.ys + (ct / kCT) * (2 * E);
    const bool in = ct < c_end;
#pragma unroll
    for (int v = 0; v < FPT; ++v) {
      const int e = threadIdx.x + v * kThreads;
      if (e < E) {
        hbuf[v] = in ? src[e] : make_uint4(0u, 0u, 0u, 0u);
        lbuf[v] = in ? src[E + e] : make_uint4(0u, 0u, 0u, 0u);
      }
    }
    if (threadIdx.x < kCT) {
      const float* xt = a.xc + ct * a.xc_stride;
      const int o = (int)threadIdx.x * a.xc_stride;
      if ((int64_t)threadIdx.x < c_end - ct)
        xbuf = make_float4(xt[o], xt[o + 1], xt[o + 2], 0.f);
      else
        xbuf = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int v = 0; v < FPT; ++v) {
      const int e = threadIdx.x + v * kThreads;
      if (e < E) {
        s_yh[buf][e] = hbuf[v];
        s_yl[buf][e] = lbuf[v];
      }
    }
    if (threadIdx.x < kCT) s_x[buf][threadIdx.x] = gram_column(xbuf, a.coord_scale, cx, cy, cz);
  };

  int buf = 0;
  fetch(c_begin);
  stash(0);
  __syncthreads();
  for (int64_t cg = c_begin; cg < c_end; cg += kFlushTiles * kCT) {
#pragma unroll
    for (int f = 0; f < kFlushTiles; ++f) {
      const int64_t ct = cg + f * kCT;
      fetch(ct + kCT);
      const float* sxf = reinterpret_cast<const float*>(&s_x[buf][0]);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int m = lane & 15;
        const int col = ks * 32 + 8 * (m >> 2) + (m & 3);
        const float ad0 = sxf[4 * col + (lane >> 4)];
        const float ad1 = sxf[4 * (col + 4) + (lane >> 4)];
        bf8v yh[NT], yl[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          yh[t] = __builtin_bit_cast(bf8v, s_yh[buf][(ks * NT + t) * 64 + lane]);
          yl[t] = __builtin_bit_cast(bf8v, s_yl[buf][(ks * NT + t) * 64 + lane]);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const f4v d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ad0, bx[rb], zero4, 0, 0, 0);
          const f4v d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ad1, bx[rb], zero4, 0, 0, 0);
          float g[8];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            g[u] = __builtin_amdgcn_exp2f(d0[u]);
            g[4 + u] = __builtin_amdgcn_exp2f(d1[u]);
          }
          uint4 gh, gl;
          split2(g[0], g[1], gh.x, gl.x);
          split2(g[2], g[3], gh.y, gl.y);
          split2(g[4], g[5], gh.z, gl.z);
          split2(g[6], g[7], gh.w, gl.w);
          const bf8v ah = __builtin_bit_cast(bf8v, gh);
          const bf8v al = __builtin_bit_cast(bf8v, gl);
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            acc[rb][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, yh[t], acc[rb][t], 0, 0, 0);
            acc[rb][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, yl[t], acc[rb][t], 0, 0, 0);
            acc[rb][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, yh[t], acc[rb][t], 0, 0, 0);
          }
        }
      }
      stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
    flush();
  }

  float* out = a.nsplit > 1 ? a.partial + (size_t)split * a.nr * B : a.Z;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + 16 * rb + 4 * (lane >> 4) + r;
      if (row < a.nr) {
        const float sc = a.out_scale * (a.rs ? a.rs[row] : 1.0f);
        const double f = sc * gram_row_factor(a, row, cx, cy, cz);
#pragma unroll
        for (int t = 0; t < NT; ++t) out[row * B + 16 * t + (lane & 15)] = (float)(f * tot[rb][t][r]);
      }
    }
  }
}

// One BF16x3 work item: the Gram form where it applies, else the difference
// form.
template <int KERNEL, int B, int RB>
__device__ __forceinline__ void gamma_bf16x3_item(const GammaLaunch& a, int64_t rblk, int split, float4 (*s_x)[kCT],
                                                  uint4 (*s_yh)[kKS * (B / 16) * 64],
                                                  uint4 (*s_yl)[kKS * (B / 16) * 64], float (*s_box)[8]) {
  if constexpr (KERNEL == KA_GAUSSIAN) {
    float cx, cy, cz;
    if (gram_rows<RB>(a, rblk, s_box, cx, cy, cz)) {
      gamma_bf16x3_gram_tile<B, RB>(a, rblk, split, s_x, s_yh, s_yl, cx, cy, cz);
      return;
    }
  }
  gamma_bf16x3_tile<KERNEL, B, RB>(a, rblk, split, s_x, s_yh, s_yl);
}

// Occupancy target of the BF16x3 path (waves per SIMD), measured best on the
// workload shapes: 4 at b = 16, 3 at b = 32 and 64.  At b = 64 the Gaussian
// kernel's Gram-form tile runs 23% faster at 3 than at 2; the difference-form
// tile beside it, taken only by wide row blocks, then spills (4 scratch
// accesses per two tiles in its loop).
template <int B>
constexpr int bf16x3_waves() { return B == 16 ? 4 : 3; }

template <int KERNEL, int B, int RB>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(bf16x3_waves<B>(), bf16x3_waves<B>())))
void gamma_bf16x3_kernel(GammaLaunch a) {
  __shared__ float4 s_x[2][kCT];
  __shared__ uint4 s_yh[2][kKS * (B / 16) * 64];
  __shared__ uint4 s_yl[2][kKS * (B / 16) * 64];
  __shared__ float s_box[4][8];
  int64_t rblk;
  int split;
  if (!gamma_item(a, rblk, split)) return;
  gamma_bf16x3_item<KERNEL, B, RB>(a, rblk, split, s_x, s_yh, s_yl, s_box);
}

// Several kernel products in one persistent launch: work items (product,
// row block, column split) are taken round-robin by the workgroups.  Each
// product keeps its own split-K partition, so its result does not depend on
// what else is in the batch.
// The batched kernel inlines the tiles of both kernel functions and its item
// loop, so it needs more registers than a single-product launch: 3 waves per
// SIMD at b = 16 and 2 at b = 32 and 64 keep it free of spills.
template <int B, int PREC>
constexpr int batch_waves() { return B == 16 ? 3 : 2; }

template <int B, int RB, int PREC>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(batch_waves<B, PREC>(), batch_waves<B, PREC>())))
void gamma_batch_kernel(const GammaJob* __restrict__ jobs,
                                                               const GammaItem* __restrict__ items, int n_items) {
  __shared__ float4 s_x[2][kCT];
  __shared__ float s_y[PREC == KA_FP32 ? 2 : 1][PREC == KA_FP32 ? kCT * y_stride<B>() : 1];
  __shared__ uint4 s_yh[PREC == KA_FP32 ? 1 : 2][PREC == KA_FP32 ? 1 : kKS * (B / 16) * 64];
  __shared__ uint4 s_yl[PREC == KA_FP32 ? 1 : 2][PREC == KA_FP32 ? 1 : kKS * (B / 16) * 64];
  __shared__ float s_box[4][8];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const GammaItem item = items[it];
    const GammaLaunch a = jobs[item.job].a;
    const int kernel = jobs[item.job].kernel;
    if constexpr (PREC == KA_FP32) {
      auto sy = reinterpret_cast<float(*)[kCT * y_stride<B>()]>(&s_y[0][0]);
      if (kernel == KA_GAUSSIAN) gamma_f32_item<KA_GAUSSIAN, B, RB>(a, item.rblk, item.split, s_x, sy, s_box);
      else gamma_f32_tile<KA_EXP_L1, B, RB>(a, item.rblk, item.split, s_x, sy);
    } else {
      auto yh = reinterpret_cast<uint4(*)[kKS * (B / 16) * 64]>(&s_yh[0][0]);
      auto yl = reinterpret_cast<uint4(*)[kKS * (B / 16) * 64]>(&s_yl[0][0]);
      if (kernel == KA_GAUSSIAN) gamma_bf16x3_item<KA_GAUSSIAN, B, RB>(a, item.rblk, item.split, s_x, yh, yl, s_box);
      else gamma_bf16x3_tile<KA_EXP_L1, B, RB>(a, item.rblk, item.split, s_x, yh, yl);
    }
    __syncthreads();
  }
}

// BF16x3 pre-pass of a batched launch: job blockIdx.y splits its own Y.
template <int B>
__global__ __launch_bounds__(256) void gamma_split_jobs_kernel(const GammaJob* __restrict__ jobs) {
  const GammaLaunch& a = jobs[blockIdx.y].a;
  const int64_t n = split_entries<B>(a.nc);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    split_y_entry<B>(a.Y, a.nc, a.ys, e);
}

// Sum of split-K partials in fixed order: Z = sum_s partial[s].
__global__ void gamma_reduce_kernel(const float* __restrict__ partial, int nsplit, int64_t n,
                                    float* __restrict__ Z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += partial[(size_t)k * n + i];
  Z[i] = (float)s;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int rows_per_block(int b, int precision) {
  (void)precision;
  return 4 * 16 * (b == 64 ? 2 : 4);
}

constexpr int64_t kMinSplitCols = 512;

GammaPlan gamma_plan(int64_t nr, int64_t nc, int b, int precision) {
  GammaPlan p;
  p.rows_per_block = rows_per_block(b, precision);
  p.row_blocks = (nr + p.rows_per_block - 1) / p.rows_per_block;
  p.xcd_splits = 0;
  if (nr <= 0 || nc <= 0) {   // nothing to split
    p.nsplit = 1;
    p.cols_per_split = nc > 0 ? nc : 0;
    p.partial_bytes = 0;
    p.ysplit_bytes = 0;
    p.work_bytes = 0;
    return p;
  }
  // Fill the chip: aim for >= 2048 workgroups, but keep >= kMinSplitCols
  // columns per split so the partial-sum traffic stays small next to the pair
  // work (a split's partial sums are b floats per row; its pairs are
  // kMinSplitCols per row at least).
  const int64_t target = 2048;
  int64_t ns = (target + p.row_blocks - 1) / p.row_blocks;
  const int64_t max_by_cols = nc / kMinSplitCols;
  if (ns > max_by_cols) ns = max_by_cols;
  if (ns > 64) ns = 64;
  if (ns < 1) ns = 1;
  // L2 fit.  With fewer than 8 splits every XCD streams every split's column
  // range, and a range larger than an XCD's L2 (4 MB) is then re-read from
  // HBM by each round of workgroups.  Eight or more XCD-grouped splits of at
  // most kL2FitBytes each are fetched about once, at the price of more
  // partial sums; taken when those cost fewer bytes than one re-read of the
  // columns per XCD.
  const double col_bytes = 16.0 + 4.0 * b;   // a point (float4) and its row of Y
  if (ns < kXcds && (double)nc * col_bytes / ns > kL2FitBytes) {
    int64_t ns2 = kXcds;
    while ((double)((nc + ns2 - 1) / ns2) * col_bytes > kL2FitBytes && ns2 + kXcds <= 64) ns2 += kXcds;
    if (ns2 <= max_by_cols && (double)ns2 * nr * b * 4 < (double)nc * col_bytes * kXcds) ns = ns2;
  }
  // With at least one split per XCD, round the split count up to a multiple
  // of the XCD count: the grouped grid then keeps every split on one XCD, so
  // its column range is fetched from HBM into that XCD's L2 once.
  if (ns >= kXcds) ns = (ns + kXcds - 1) / kXcds * kXcds;
  // Whole tile groups per split: only the last split can end in a padding tile.
  int64_t cps = (nc + ns - 1) / ns;
  cps = (cps + kFlushTiles * kCT - 1) / (kFlushTiles * kCT) * (kFlushTiles * kCT);
  const int64_t ns_grid = ns;
  ns = (nc + cps - 1) / cps;
  if (ns < 1) ns = 1;
  p.nsplit = (int)ns;
  p.cols_per_split = cps;
  p.partial_bytes = ns > 1 ? (size_t)ns * nr * b * sizeof(float) : 0;
  p.ysplit_bytes = precision == KA_BF16X3 ? (size_t)((nc + kCT - 1) / kCT) * kCT * b * 4 : 0;
  p.work_bytes = (p.partial_bytes + 255) / 256 * 256 + p.ysplit_bytes;
  p.xcd_splits = ns_grid >= kXcds ? (int)ns_grid : 0;
  return p;
}

uint4* gamma_ysplit_ptr(float* work, const GammaPlan& p) {
  if (p.ysplit_bytes == 0 || !work) return nullptr;
  return reinterpret_cast<uint4*>(reinterpret_cast<char*>(work) + (p.partial_bytes + 255) / 256 * 256);
}

static hipError_t launch_split(const float* Y, int64_t nc, uint4* ys, int b, hipStream_t s) {
  const int64_t n = nc <= 0 ? 0 : (b == 16 ? split_entries<16>(nc) : b == 32 ? split_entries<32>(nc) : split_entries<64>(nc));
  if (n == 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  switch (b) {
    case 16: hipLaunchKernelGGL(gamma_split_kernel<16>, dim3(grid), dim3(256), 0, s, Y, nc, ys); break;
    case 32: hipLaunchKernelGGL(gamma_split_kernel<32>, dim3(grid), dim3(256), 0, s, Y, nc, ys); break;
    case 64: hipLaunchKernelGGL(gamma_split_kernel<64>, dim3(grid), dim3(256), 0, s, Y, nc, ys); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KERNEL>
static hipError_t launch_kernel_variant(const GammaLaunch& a, int b, int precision, dim3 grid,
                                        hipStream_t s) {
  if (precision == KA_FP32) {
    switch (b) {
      case 16: hipLaunchKernelGGL((gamma_f32_kernel<KERNEL, 16, 4>), grid, dim3(kThreads), 0, s, a); break;
      case 32: hipLaunchKernelGGL((gamma_f32_kernel<KERNEL, 32, 4>), grid, dim3(kThreads), 0, s, a); break;
      case 64: hipLaunchKernelGGL((gamma_f32_kernel<KERNEL, 64, 2>), grid, dim3(kThreads), 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (b) {
      case 16: hipLaunchKernelGGL((gamma_bf16x3_kernel<KERNEL, 16, 4>), grid, dim3(kThreads), 0, s, a); break;
      case 32: hipLaunchKernelGGL((gamma_bf16x3_kernel<KERNEL, 32, 4>), grid, dim3(kThreads), 0, s, a); break;
      case 64: hipLaunchKernelGGL((gamma_bf16x3_kernel<KERNEL, 64, 2>), grid, dim3(kThreads), 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_gamma(GammaLaunch a, int kernel, int b, int precision, hipStream_t s) {
  if (a.nr <= 0) return hipSuccess;
  const GammaPlan p = gamma_plan(a.nr, a.nc, b, precision);
  a.nsplit = p.nsplit;
  a.cols_per_split = p.cols_per_split;
  a.row_blocks = p.row_blocks;
  a.xcd_splits = p.xcd_splits;
  if (a.nc <= 0) {
    return fill_zero_f32(a.Z, a.nr * b, s);
  }
  if (precision == KA_BF16X3) {
    a.ys = gamma_ysplit_ptr(a.partial, p);
    if (!a.ys) return hipErrorInvalidValue;
    const hipError_t e = launch_split(a.Y, a.nc, a.ys, b, s);
    if (e != hipSuccess) return e;
  }
  const dim3 grid = p.xcd_splits > 0 ? dim3((unsigned)(p.row_blocks * p.xcd_splits), 1u)
                                     : dim3((unsigned)p.row_blocks, (unsigned)p.nsplit);
  hipError_t e = (kernel == KA_GAUSSIAN) ? launch_kernel_variant<KA_GAUSSIAN>(a, b, precision, grid, s)
                                         : launch_kernel_variant<KA_EXP_L1>(a, b, precision, grid, s);
  if (e != hipSuccess) return e;
  if (p.nsplit > 1) {
    const int64_t n = a.nr * b;
    hipLaunchKernelGGL(gamma_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       a.partial, p.nsplit, n, a.Z);
    e = hipGetLastError();
  }
  return e;
}

int gamma_rows_per_block(int b) { return rows_per_block(b, KA_FP32); }

hipError_t launch_gamma_batch(const GammaJob* jobs_dev, const GammaItem* items_dev, int n_items, int b,
                              int precision, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const int grid = n_items < 4096 ? n_items : 4096;
  if (precision == KA_FP32) {
    switch (b) {
      case 16: hipLaunchKernelGGL((gamma_batch_kernel<16, 4, KA_FP32>), dim3(grid), dim3(kThreads), 0, s, jobs_dev, items_dev, n_items); break;
      case 32: hipLaunchKernelGGL((gamma_batch_kernel<32, 4, KA_FP32>), dim3(grid), dim3(kThreads), 0, s, jobs_dev, items_dev, n_items); break;
      case 64: hipLaunchKernelGGL((gamma_batch_kernel<64, 2, KA_FP32>), dim3(grid), dim3(kThreads), 0, s, jobs_dev, items_dev, n_items); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (b) {
      case 16: hipLaunchKernelGGL((gamma_batch_kernel<16, 4, KA_BF16X3>), dim3(grid), dim3(kThreads), 0, s, jobs_dev, items_dev, n_items); break;
      case 32: hipLaunchKernelGGL((gamma_batch_kernel<32, 4, KA_BF16X3>), dim3(grid), dim3(kThreads), 0, s, jobs_dev, items_dev, n_items); break;
      case 64: hipLaunchKernelGGL((gamma_batch_kernel<64, 2, KA_BF16X3>), dim3(grid), dim3(kThreads), 0, s, jobs_dev, items_dev, n_items); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_gamma_split_jobs(const GammaJob* jobs_dev, int n_jobs, int b, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  const dim3 grid(256, (unsigned)n_jobs);
  switch (b) {
    case 16: hipLaunchKernelGGL(gamma_split_jobs_kernel<16>, grid, dim3(256), 0, s, jobs_dev); break;
    case 32: hipLaunchKernelGGL(gamma_split_jobs_kernel<32>, grid, dim3(256), 0, s, jobs_dev); break;
    case 64: hipLaunchKernelGGL(gamma_split_jobs_kernel<64>, grid, dim3(256), 0, s, jobs_dev); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gamma_reduce(const float* partial, int nsplit, int64_t n, float* Z, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gamma_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, partial, nsplit, n, Z);
  return hipGetLastError();
}

}  // namespace ka
