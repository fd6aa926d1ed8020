// FP64 dense kernels of the block eigensolver: tall-skinny products for the
// block orthogonalisation and Rayleigh-Ritz projection, Cholesky-QR of a
// block, the orthonormal basis of a set of vectors from their Gram matrix
// (pivoted Cholesky, for the collocation restart), column norms, residual
// assembly, sign normalisation and a counter-based normal
// generator for start blocks.  All reductions use a fixed partition and a
// fixed summation order, so results depend only on the shapes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "basis_core.hpp"
#include "ka_internal.hpp"

namespace ka {

__global__ void split_reduce_kernel(const double* __restrict__ part, int nsplit, int m, int n, double alpha,
                                    double beta, double* __restrict__ C, int64_t ldc) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)m * n) return;
  const int i = (int)(id % m), j = (int)(id / m);
  // four interleaved partial sums (fixed order), so several loads are in flight
  const size_t stride = (size_t)n * m;
  const double* p = part + (size_t)j * m + i;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int z = 0;
  for (; z + 3 < nsplit; z += 4) {
    s0 += p[(size_t)z * stride];
    s1 += p[(size_t)(z + 1) * stride];
    s2 += p[(size_t)(z + 2) * stride];
    s3 += p[(size_t)(z + 3) * stride];
  }
  for (; z < nsplit; ++z) s0 += p[(size_t)z * stride];
  const double s = (s0 + s1) + (s2 + s3);
  double* c = C + i + (int64_t)j * ldc;
  *c = (beta == 0.0) ? alpha * s : alpha * s + beta * *c;
}

// ---------------------------------------------------------------------------
// C = alpha A^T B + beta C for tall A (K x m) and B (K x n): the projections
// and Gram matrices of the block eigensolver (K = N up to ~10^6, m up to a
// few hundred, n the block width).  The product reads A and B once from HBM
// and does 2 K m n flops on the FP64 matrix cores; a workgroup therefore takes
// a 128 x 64 block of C, so that A is read once and B once per 128 rows of C.
//
// v_mfma_f64_16x16x4f64 layout: A lane l holds (i = l % 16, k = l / 16), B
// lane l holds (k = l / 16, j = l % 16), accumulator register r of lane l
// holds (i = l / 16 + 4 r, j = l % 16).  The four MFMAs of a 16-row step may
// take its rows in any partition, so lane l reads the four consecutive rows
// 4 (l / 16) .. + 3 of its columns of A (MFMA s takes row 4 (l / 16) + s).
// Each of the 4 waves holds two 16-row tiles of C across the block's four
// 16-column tiles (8 accumulators) and reads A straight from memory, the
// next step's rows issued before the current step's MFMAs.  B, the same for
// the 4 waves, goes through LDS in chunks of kTnStep rows (zero past the
// row range and past n, so the clamped rows of A beyond the range add
// nothing), double buffered with one barrier per chunk.  Row ranges (splits)
// go to a partial array that split_reduce_kernel sums in split order, or
// straight to C with one split.
// ---------------------------------------------------------------------------
typedef double tn_d4 __attribute__((ext_vector_type(4)));
constexpr int kTnI = 2;                     // 16-row tiles of C per wave
constexpr int kTnRowsC = 4 * 16 * kTnI;     // rows of C (columns of A) per workgroup
constexpr int kTnStep = 32;                 // rows of A and B per chunk (two 16-row steps)
constexpr int kTnBW = 64 + 8;               // padded LDS row of a B chunk (doubles)
constexpr int kTnSE = kTnStep * 64 / 256;   // staged B elements per thread

__global__ __launch_bounds__(256) void dgemm_tn_mfma_kernel(int m, int n, int64_t K, const double* __restrict__ A,
                                                            int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                            int64_t k_per_split, double* __restrict__ part,
                                                            double alpha, double beta, double* __restrict__ C,
                                                            int64_t ldc) {
  __shared__ double Bs[2][kTnStep][kTnBW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane >> 4, c16 = lane & 15;
  const int i0 = blockIdx.x * kTnRowsC + w * 16 * kTnI;   // this wave's first row of C
  const bool on = i0 < m;                                  // (a wave past m only stages B)
  const int j0 = blockIdx.y * 64;
  const double* Ap[kTnI];
#pragma unroll
  for (int u = 0; u < kTnI; ++u) {
    const int i = i0 + 16 * u + c16;
    Ap[u] = A + (int64_t)(i < m ? i : 0) * lda;
  }
  const int64_t kb = (int64_t)blockIdx.z * k_per_split;
  const int64_t ke = kb + k_per_split < K ? kb + k_per_split : K;
  tn_d4 acc[kTnI][4];
#pragma unroll
  for (int u = 0; u < kTnI; ++u)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[u][t] = (tn_d4){0.0, 0.0, 0.0, 0.0};
  double st[kTnSE];
  auto fetch_b = [&](int64_t g) {            // consecutive threads down a column of B
#pragma unroll
    for (int v = 0; v < kTnSE; ++v) {
      const int e = threadIdx.x + 256 * v;
      const int64_t r = g + e % kTnStep;
      const int j = j0 + e / kTnStep;
      st[v] = (r < ke && j < n) ? B[r + (int64_t)j * ldb] : 0.0;
    }
  };
  auto put_b = [&](int buf) {
#pragma unroll
    for (int v = 0; v < kTnSE; ++v) {
      const int e = threadIdx.x + 256 * v;
      Bs[buf][e % kTnStep][e / kTnStep] = st[v];
    }
  };
  // one 16-row step of A; rows past the range are read at row ke - 1 (a
  // valid address) and meet zeros of B
  auto load_a = [&](int64_t g, double (&a)[kTnI][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t r = g + 4 * q + s;
      const int64_t rc = r < ke ? r : ke - 1;
#pragma unroll
      for (int u = 0; u < kTnI; ++u) a[u][s] = Ap[u][rc];
    }
  };
  auto step = [&](int buf, int h, const double (&a)[kTnI][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[t] = Bs[buf][16 * h + 4 * q + s][16 * t + c16];
#pragma unroll
      for (int u = 0; u < kTnI; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[u][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][s], bv[t], acc[u][t], 0, 0, 0);
    }
  };
  if (kb < ke) {                             // uniform over the workgroup, like every branch below
    double a0[kTnI][4], a1[kTnI][4];
    fetch_b(kb);
    put_b(0);
    load_a(kb, a0);
    __syncthreads();
    int buf = 0;
    for (int64_t g = kb; g < ke; g += kTnStep) {
      const bool more = g + kTnStep < ke;
      if (more) fetch_b(g + kTnStep);
      load_a(g + 16, a1);
      if (on) step(buf, 0, a0);
      if (more) load_a(g + kTnStep, a0);
      if (on) step(buf, 1, a1);
      if (more) put_b(buf ^ 1);              // its last readers finished before the previous barrier
      __syncthreads();
      buf ^= 1;
    }
  }
  if (!on) return;
#pragma unroll
  for (int u = 0; u < kTnI; ++u)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int jo = j0 + 16 * t + c16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int io = i0 + 16 * u + q + 4 * r;
        if (io >= m || jo >= n) continue;
        const double v = acc[u][t][r];
        if (part) {
          part[((size_t)blockIdx.z * n + jo) * m + io] = v;   // partial[z][j][i]
        } else {
          double* c = C + io + (int64_t)jo * ldc;
          *c = (beta == 0.0) ? alpha * v : alpha * v + beta * *c;
        }
      }
    }
}

// Row splits: about 512 workgroups (two per CU), at least 256 rows each,
// whole multiples of kTnStep, at most 256 splits; products with K < 1024
// take one split.
static int64_t tn_rows_per_split(int m, int n, int64_t K) {
  if (K < 1024) return K > 0 ? K : 1;
  const int64_t tiles = (int64_t)((m + kTnRowsC - 1) / kTnRowsC) * ((n + 63) / 64);
  int64_t ns = (512 + tiles - 1) / tiles;
  if (ns > K / 256) ns = K / 256;
  if (ns > 256) ns = 256;
  if (ns < 1) ns = 1;
  const int64_t kps = (K + ns - 1) / ns;
  return (kps + kTnStep - 1) / kTnStep * kTnStep;
}

static int tn_splits(int m, int n, int64_t K) {
  const int64_t kps = tn_rows_per_split(m, n, K);
  return K > 0 ? (int)((K + kps - 1) / kps) : 1;
}

size_t dgemm_tn_work(int m, int n, int64_t K) {
  const int ns = tn_splits(m, n, K);
  return ns > 1 ? (size_t)ns * m * n : 0;
}

hipError_t dgemm_tn(int m, int n, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
                    int64_t ldb, double beta, double* C, int64_t ldc, double* work, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t kps = tn_rows_per_split(m, n, K);
  const int ns = tn_splits(m, n, K);
  const dim3 grid((m + kTnRowsC - 1) / kTnRowsC, (n + 63) / 64, ns);
  hipLaunchKernelGGL(dgemm_tn_mfma_kernel, grid, dim3(256), 0, s, m, n, K, A, lda, B, ldb, kps,
                     ns > 1 ? work : nullptr, alpha, beta, C, ldc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ns == 1) return e;
  const int64_t tot = (int64_t)m * n;
  hipLaunchKernelGGL(split_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, work, ns, m, n,
                     alpha, beta, C, ldc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// C = alpha A B + beta C for tall A (M x k) and small B (k x n): basis
// updates X C, restarts X S and the Cholesky-QR step of the block
// eigensolver (M = N, k and n up to a few hundred).
//
// A workgroup computes 64 rows x 128 columns of C: wave w holds rows
// 16 w .. 16 w + 15 across eight 16-column MFMA tiles (the MFMA layout of the
// A^T B kernel above: lane l of the A operand reads A at row l % 16 and
// column 4 s + l / 16, so 16 lanes read 128 contiguous bytes).  B goes through
// LDS in chunks of 32 rows, stored row-major with a padded row so that a
// fragment read (4 rows x 16 columns) touches every bank twice, the least a
// 64-lane FP64 read can.  While a chunk's MFMAs run, the next chunk of B and
// the next 8 A values per lane are already loading.
// ---------------------------------------------------------------------------
// 64 x 64 blocks of C: a small accumulator and LDS footprint let 4 waves
// share each SIMD to hide the load latency of A (measured against 64 x 128
// blocks at 2 waves per SIMD, N = 287,496: 0.22 against 0.35 ms per call on
// average over the orthogonalisation products (n = 64, k up to 456), and 2.47
// against 2.89 ms at n = 264, k = 456)
constexpr int kNnJ = 4;                      // 16-column tiles per workgroup
constexpr int kNnKC = 32;                    // rows of B per LDS chunk
constexpr int kNnBW = 16 * kNnJ + 16;        // padded LDS row of B (doubles)
constexpr int kNnSE = kNnKC * 16 * kNnJ / 256;   // staged B elements per thread

// Grid: 1-D, the row blocks rounded up to a multiple of 8 times the column
// blocks.  Workgroup L runs on XCD L % 8; on each XCD the column blocks of a
// row block follow one another, so the block's 64 rows of A are read from HBM
// about once and then from that XCD's L2 (with the column blocks outermost,
// A was read from HBM once per column block).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
void dgemm_nn_mfma_kernel(int64_t M, int n, int k, const double* __restrict__ A, int64_t lda,
                          const double* __restrict__ B, int64_t ldb, double alpha, double beta,
                          double* __restrict__ C, int64_t ldc) {
  __shared__ double Bs[2][kNnKC][kNnBW];
  const int ncb = (n + 16 * kNnJ - 1) / (16 * kNnJ);
  const int64_t L = blockIdx.x, seq = L / 8;
  const int64_t rb = (seq / ncb) * 8 + L % 8;   // row block
  const int cb = (int)(seq % ncb);              // column block
  if (rb * 64 >= M) return;                     // padding workgroup (whole workgroup)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane >> 4, c16 = lane & 15;
  const int64_t r0 = rb * 64 + 16 * w;
  const int64_t i = r0 + c16;
  const bool iok = i < M;
  const double* __restrict__ Ai = A + (iok ? i : M - 1);
  const int j0 = cb * 16 * kNnJ;
  const int jt = (n - j0 + 15) / 16 < kNnJ ? (n - j0 + 15) / 16 : kNnJ;   // column tiles of this workgroup
  const int nch = (k + kNnKC - 1) / kNnKC;
  tn_d4 acc[kNnJ];
#pragma unroll
  for (int t = 0; t < kNnJ; ++t) acc[t] = (tn_d4){0.0, 0.0, 0.0, 0.0};
  double st[kNnSE];
  auto fetch_b = [&](int c) {                // chunk c of B (zeros past k and n), consecutive threads down a column
#pragma unroll
    for (int v = 0; v < kNnSE; ++v) {
      const int e = threadIdx.x + 256 * v;
      const int kk = c * kNnKC + e % kNnKC, j = j0 + e / kNnKC;
      st[v] = (kk < k && j < n) ? B[kk + (int64_t)j * ldb] : 0.0;
    }
  };
  auto put_b = [&](int buf) {
#pragma unroll
    for (int v = 0; v < kNnSE; ++v) {
      const int e = threadIdx.x + 256 * v;
      Bs[buf][e % kNnKC][e / kNnKC] = st[v];
    }
  };
  double a[kNnKC / 4], an[kNnKC / 4];
  auto fetch_a = [&](int c, double (&x)[kNnKC / 4]) {   // rows past k are read at row k - 1 and weighted by zero
#pragma unroll
    for (int s = 0; s < kNnKC / 4; ++s) {
      const int kk = c * kNnKC + 4 * s + q;
      x[s] = k > 0 ? Ai[(int64_t)(kk < k ? kk : k - 1) * lda] : 0.0;
    }
  };
  fetch_b(0);
  put_b(0);
  fetch_a(0, a);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {            // uniform over the workgroup
    const int buf = c & 1;
    if (c + 1 < nch) {
      fetch_b(c + 1);
      fetch_a(c + 1, an);
    }
#pragma unroll
    for (int s = 0; s < kNnKC / 4; ++s) {
      const int kk = c * kNnKC + 4 * s + q;
      const double av = (kk < k && iok) ? a[s] : 0.0;
#pragma unroll
      for (int t = 0; t < kNnJ; ++t)
        if (t < jt)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bs[buf][4 * s + q][16 * t + c16], acc[t], 0, 0, 0);
    }
    if (c + 1 < nch) {
      put_b(buf ^ 1);                        // the other buffer: its last readers finished before the barrier
#pragma unroll
      for (int s = 0; s < kNnKC / 4; ++s) a[s] = an[s];
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < kNnJ; ++t) {
    const int jo = j0 + 16 * t + c16;
    if (t >= jt || jo >= n) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t io = r0 + q + 4 * r;
      if (io >= M) continue;
      double* cp = C + io + (int64_t)jo * ldc;
      *cp = (beta == 0.0) ? alpha * acc[t][r] : alpha * acc[t][r] + beta * *cp;
    }
  }
}

hipError_t dgemm_nn(int64_t M, int n, int k, double alpha, const double* A, int64_t lda, const double* B,
                    int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s) {
  if (M <= 0 || n <= 0) return hipSuccess;
  const int64_t nrb8 = ((M + 63) / 64 + 7) / 8 * 8;
  const int64_t ncb = (n + 16 * kNnJ - 1) / (16 * kNnJ);
  if (nrb8 * ncb > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(nrb8 * ncb), 1, 1);
  hipLaunchKernelGGL(dgemm_nn_mfma_kernel, grid, dim3(256), 0, s, M, n, k, A, lda, B, ldb, alpha, beta, C, ldc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cholesky of a small SPD Gram matrix G = R^T R and R^-1 (upper), n <= 64.
// status: 0 ok, 1 a pivot was not positive or lost (rank-deficient block).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void chol_upper_inv_kernel(const double* __restrict__ G, int n, int ldg,
                                                            double* __restrict__ Rinv, int ldr, int* status,
                                                            const double* __restrict__ ref) {
  __shared__ double R[64][65];
  __shared__ double X[64][65];
  __shared__ int bad;
  __shared__ double piv;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int i = 0; i < n; ++i) R[i][t] = (t < n) ? G[i + t * ldg] : 0.0;   // R holds G (symmetric)
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    // row j of R: R[j][j] = sqrt(G_jj - sum_k R_kj^2), R[j][i] = (G_ji - sum_k R_kj R_ki) / R_jj
    if (t == 0) {
      double d = R[j][j];
      for (int k = 0; k < j; ++k) d -= R[k][j] * R[k][j];
      const double orig = G[j + j * ldg];
      const double floor = ref ? kOrthKeep * kOrthKeep * ref[j] * ref[j] : 0.0;
      if (!(d > 1e-26 * orig) || !(orig > 1e-300) || !(d > floor)) {
        bad = 1;
        d = 1.0;
      }
      piv = sqrt(d);
    }
    __syncthreads();
    if (t > j && t < n) {
      double sv = R[j][t];
      for (int k = 0; k < j; ++k) sv -= R[k][j] * R[k][t];
      R[j][t] = sv / piv;
    }
    __syncthreads();
    if (t == 0) R[j][j] = piv;
    __syncthreads();
  }
  // zero strict lower part (it held G)
  for (int i = 0; i < n; ++i)
    if (t < i) R[i][t] = 0.0;
  __syncthreads();
  // X = R^-1, column t by back substitution: R x = e_t
  if (t < n) {
    for (int i = n - 1; i >= 0; --i) {
      double sv = (i == t) ? 1.0 : 0.0;
      for (int k = i + 1; k < n; ++k) sv -= R[i][k] * X[k][t];
      X[i][t] = (i > t) ? 0.0 : sv / R[i][i];
    }
  }
  __syncthreads();
  for (int i = 0; i < n; ++i)
    if (t < n) Rinv[i + t * ldr] = X[i][t];
  if (t == 0) *status = bad;
}

hipError_t chol_upper_inv(const double* G, int n, int ldg, double* Rinv, int ldr, int* status, hipStream_t s,
                          const double* ref) {
  if (n > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_upper_inv_kernel, dim3(1), dim3(64), 0, s, G, n, ldg, Rinv, ldr, status, ref);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Orthonormal basis of span(S) from its Gram matrix G = S^T S (n x n, n at
// most the Rayleigh-Ritz order): diagonal-pivoted Cholesky with a rank cut and
// the inverse of its factor (basis_core.hpp), one workgroup, working copy in
// LDS up to order kBasisLds.  W (n x rank, leading dimension ldw) = P R^-1;
// rank goes to a device int.
// ---------------------------------------------------------------------------
constexpr int kBasisThreads = 1024;

struct BasisTeam {
  double* rv;   // one slot per wave
  int* ri;
  __device__ int tid() const { return threadIdx.x; }
  __device__ int size() const { return kBasisThreads; }
  __device__ void sync() const { __syncthreads(); }
  // index of the largest v (smallest index among equals; -1 if none has one)
  __device__ static bool better(double v, int i, double bv, int bi) {
    return i >= 0 && (bi < 0 || v > bv || (v == bv && i < bi));
  }
  __device__ int argmax(double v, int i) const {
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(v, off);
      const int oi = __shfl_xor(i, off);
      if (better(ov, oi, v, i)) {
        v = ov;
        i = oi;
      }
    }
    if ((threadIdx.x & 63) == 0) {
      rv[threadIdx.x >> 6] = v;
      ri[threadIdx.x >> 6] = i;
    }
    __syncthreads();
    double bv = rv[0];
    int bi = ri[0];
    for (int w = 1; w < kBasisThreads / 64; ++w)
      if (better(rv[w], ri[w], bv, bi)) {
        bv = rv[w];
        bi = ri[w];
      }
    __syncthreads();
    return bi;
  }
};

// the working copy in LDS up to order kBasisLds, else in `work`
constexpr int kBasisLds = 136;
static_assert((kBasisLds * kBasisLds + 2 * kBasisLds) * 8 + (kBasisThreads / 64) * 12 <= 160 * 1024,
              "the LDS variant of the basis kernel fits in 160 KiB");

template <bool LDS>
__global__ __launch_bounds__(kBasisThreads) void pchol_basis_kernel(const double* __restrict__ G, int n, int ldg,
                                                                    double cut, double* __restrict__ work,
                                                                    double* __restrict__ W, int ldw,
                                                                    int* __restrict__ rank) {
  __shared__ double rv[kBasisThreads / 64];
  __shared__ int ri[kBasisThreads / 64];
  __shared__ double w_lds[LDS ? kBasisLds * kBasisLds + 2 * kBasisLds : 1];
  BasisTeam tm{rv, ri};
  const int r = pchol_basis(tm, G, ldg, n, cut, LDS ? w_lds : work, W, ldw);
  if (threadIdx.x == 0) *rank = r;
}

size_t basis_work(int n) { return pchol_basis_work(n); }

hipError_t orthonormal_basis(const double* G, int n, int ldg, double cut, double* W, int ldw, double* work,
                             int* rank, hipStream_t s) {
  if (n < 0 || ldg < n || ldw < n) return hipErrorInvalidValue;
  if (n <= kBasisLds)
    hipLaunchKernelGGL(pchol_basis_kernel<true>, dim3(1), dim3(kBasisThreads), 0, s, G, n, ldg, cut, work, W, ldw,
                       rank);
  else
    hipLaunchKernelGGL(pchol_basis_kernel<false>, dim3(1), dim3(kBasisThreads), 0, s, G, n, ldg, cut, work, W, ldw,
                       rank);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// column norms (two-stage, fixed order)
// ---------------------------------------------------------------------------
constexpr int kNormChunk = 4096;

size_t column_norms_work(int64_t N, int n) { return (size_t)((N + kNormChunk - 1) / kNormChunk) * n; }

__global__ __launch_bounds__(256) void colnorm_partial_kernel(const double* __restrict__ X, int64_t N,
                                                              int64_t ldx, double* __restrict__ part) {
  __shared__ double red[256];
  const int j = blockIdx.y;
  const int64_t c0 = (int64_t)blockIdx.x * kNormChunk;
  double s = 0.0;
  for (int64_t i = c0 + threadIdx.x; i < c0 + kNormChunk && i < N; i += 256) {
    const double v = X[i + (int64_t)j * ldx];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)j * gridDim.x + blockIdx.x] = red[0];
}

__global__ void colnorm_final_kernel(const double* __restrict__ part, int nchunk, int n, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t)j * nchunk + c];
  out[j] = sqrt(s);
}

hipError_t column_norms(const double* X, int64_t N, int n, int64_t ldx, double* out, double* work, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nchunk = (int)((N + kNormChunk - 1) / kNormChunk);
  hipLaunchKernelGGL(colnorm_partial_kernel, dim3(nchunk, n), dim3(256), 0, s, X, N, ldx, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colnorm_final_kernel, dim3((n + 63) / 64), dim3(64), 0, s, work, nchunk, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// misc elementwise
// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based hash.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void fill_normal_kernel(double* X, int64_t N, int n, int64_t ldx, uint64_t seed, uint64_t counter) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N * n) return;
  const int64_t i = id % N, j = id / N;
  const uint64_t key = splitmix64(seed ^ splitmix64(counter + 0x632BE59BD9B4E019ull * (uint64_t)j));
  const uint64_t h1 = splitmix64(key + 2 * (uint64_t)i), h2 = splitmix64(key + 2 * (uint64_t)i + 1);
  const double u1 = ((h1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
  X[i + j * ldx] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);   // Box-Muller
}

hipError_t fill_normal(double* X, int64_t N, int n, int64_t ldx, uint64_t seed, uint64_t counter, hipStream_t s) {
  const int64_t tot = N * n;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_normal_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, N, n, ldx, seed,
                     counter);
  return hipGetLastError();
}

__global__ void copy_cols_kernel(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t N, int n) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N * n) return;
  const int64_t i = id % N, j = id / N;
  Y[i + j * ldy] = X[i + j * ldx];
}

hipError_t copy_cols(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t N, int n, hipStream_t s) {
  const int64_t tot = N * n;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, ldx, Y, ldy, N, n);
  return hipGetLastError();
}

// R = A X s - lambda X s for real and complex-pair Ritz values.
__global__ void residual_kernel(const double* AXS, const double* XS, int64_t N, int n, int64_t ld, const double* wr,
                                const double* wi, double* R) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N * n) return;
  const int64_t i = id % N;
  const int j = (int)(id / N);
  const double lr = wr[j], li = wi ? wi[j] : 0.0;
  double r = AXS[i + j * ld] - lr * XS[i + j * ld];
  if (li > 0.0 && j + 1 < n) r += li * XS[i + (j + 1) * ld];        // real part of a pair
  else if (li < 0.0 && j > 0) r += li * XS[i + (j - 1) * ld];       // imaginary part: - |li| x_r
  R[i + j * ld] = r;
}

hipError_t residual_combine(const double* AXS, const double* XS, int64_t N, int n, int64_t ld, const double* wr,
                            const double* wi, double* R, hipStream_t s) {
  const int64_t tot = N * n;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(residual_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, AXS, XS, N, n, ld, wr,
                     wi, R);
  return hipGetLastError();
}

// sign: make the first largest-magnitude entry of each column positive
__global__ __launch_bounds__(256) void sign_fix_kernel(double* V, int64_t N, int64_t ld, const double* wi) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int j = blockIdx.x;
  if (wi && wi[j] != 0.0) return;   // parts of a complex pair keep their joint phase
  double best = -1.0;
  int64_t besti = 0;
  for (int64_t i = threadIdx.x; i < N; i += 256) {
    const double a = fabs(V[i + j * ld]);
    if (a > best) { best = a; besti = i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = besti;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double o = bv[threadIdx.x + w];
      const int64_t oi = bi[threadIdx.x + w];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const bool neg = V[bi[0] + j * ld] < 0.0;
  if (neg)
    for (int64_t i = threadIdx.x; i < N; i += 256) V[i + j * ld] = -V[i + j * ld];
}

hipError_t sign_fix(double* V, int64_t N, int n, int64_t ld, const double* wi, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sign_fix_kernel, dim3(n), dim3(256), 0, s, V, N, ld, wi);
  return hipGetLastError();
}

__global__ void scale_cols_kernel(double* V, int64_t N, int n, int64_t ld, const double* scale) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N * n) return;
  const int64_t i = id % N;
  const int j = (int)(id / N);
  V[i + j * ld] *= scale[j];
}

hipError_t scale_cols(double* V, int64_t N, int n, int64_t ld, const double* scale, hipStream_t s) {
  const int64_t tot = N * n;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, V, N, n, ld, scale);
  return hipGetLastError();
}

__global__ void scale_rows_kernel(double* V, int64_t N, int n, int64_t ld, const double* scale) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N * n) return;
  const int64_t i = id % N;
  const int j = (int)(id / N);
  V[i + j * ld] *= scale[i];
}

hipError_t scale_rows(double* V, int64_t N, int n, int64_t ld, const double* scale, hipStream_t s) {
  const int64_t tot = N * n;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_rows_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, V, N, n, ld, scale);
  return hipGetLastError();
}

__global__ void fill_zero_f32_kernel(float* p, int64_t n) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) p[id] = 0.f;
}

hipError_t fill_zero_f32(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace ka
