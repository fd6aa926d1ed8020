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
  // groups of the multishift sweep: the waves, ordered among their own
  // threads by a wavefront-scope fence (one wave's LDS operations complete in
  // issue order)
  __device__ int gsize() const { return 64; }
  __device__ int group() const { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
  __device__ void gsync() const { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }
  __device__ double gpick(double v, int src) const {      // v of lane src (src uniform in the wave)
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
  }
  __device__ int imax(int x) const {
    for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off));
    if (NT == 64) return x;
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = (double)x;
    __syncthreads();
    int s = x;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s = max(s, (int)red[w]);
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
  ns_hessenberg<LDS ? 2 : 8>(tm, A, ld, n, ws.hsub, ws.beta, v, w);
  if (LDS)
    for (int j = 0; j < n; ++j)
      for (int i = threadIdx.x; i < n; i += kNsThreads) ws.A[i + (size_t)j * n] = A[i + (size_t)j * ld];
}

// ---- eigenvalue QR by one wave, matrix in LDS --------------------------------------------
// The Francis double-shift iteration of ns_qr_values (nonsym_core.hpp, the
// same arithmetic), arranged for the 64 lanes of one wave:
//  - the two searches of each iteration (the negligible sub-diagonal that
//    splits the active window, and the start m of the double step) test 64
//    positions at once and take the first hit with a ballot, instead of a
//    serial scan with one LDS round trip per position;
//  - in the bulge chase each lane keeps the column update's new values of
//    column k in registers, and the next step reads its reflector input
//    (rows k+1..k+3 of that column) with readlane instead of through LDS;
//  - the loads of an update phase are issued together, then the arithmetic,
//    then the stores.
// LDS operations of one wave complete in issue order, so ordering between
// the phases needs only a compiler fence at wavefront scope (no wait).
constexpr int kNsQrIt = (kNsBandLds + 63) / 64;   // lane iterations over a window of <= kNsBandLds

// s_waitcnt operand with lgkmcnt = 0 and the other counters at their
// maximum (no wait): all LDS operations of the wave have completed
constexpr int kNsWaitLds = 0xC07F;

__device__ inline void ns_wave_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ inline double ns_readlane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// value of row index `idx` (relative to the window start) from the registers
// c0, c1, c2 (row idx, idx - 64, idx - 128) of lane idx % 64; named scalars,
// so the selection stays in registers
static_assert(kNsQrIt == 3, "the register selection below covers three lane iterations");
__device__ inline double ns_lane_value(double c0, double c1, double c2, int idx) {
  const int it = idx >> 6;
  const double v = it == 0 ? c0 : (it == 1 ? c1 : c2);
  return ns_readlane(v, idx & 63);
}

// Inlined, so that each call site reads its band with LDS instructions.
__device__ KA_FORCEINLINE int ns_qr_values_wave(double* hb, int n, double* wr, double* wi, double* anorm_out,
                                                double tol = kNsEps) {
  const int t = threadIdx.x;
#define HB(i, j) hb[(j) * ((j) + 7) / 2 + (i)]
  double anorm = 0.0;
  for (int j = t; j < n; j += 64)
    for (int i = 0; i <= j + 1 && i < n; ++i) anorm += fabs(HB(i, j));
  for (int off = 32; off > 0; off >>= 1) anorm += __shfl_xor(anorm, off);
  if (anorm_out && t == 0) *anorm_out = anorm;
  int nn = n - 1;
  double shift = 0.0;
  int fail = 0;
  while (nn >= 0 && !fail) {
    int its = 0;
    while (true) {
      ns_wave_fence();
      // largest l in [1, nn] with a negligible sub-diagonal H(l, l-1), else 0
      int l = 0;
      for (int base = nn; base >= 1; base -= 64) {
        const int l0 = base - t;
        bool hit = false;
        if (l0 >= 1) {
          double s = fabs(HB(l0 - 1, l0 - 1)) + fabs(HB(l0, l0));
          if (s == 0.0) s = anorm;
          hit = fabs(HB(l0, l0 - 1)) <= tol * s;
        }
        const unsigned long long mask = __ballot(hit);
        if (mask) {
          l = base - (__ffsll(mask) - 1);
          break;
        }
      }
      double x = HB(nn, nn);
      if (l == nn) {                                   // one real eigenvalue
        if (t == 0) {
          wr[nn] = x + shift;
          wi[nn] = 0.0;
        }
        --nn;
        break;
      }
      double y = HB(nn - 1, nn - 1);
      double w = HB(nn, nn - 1) * HB(nn - 1, nn);
      if (l == nn - 1) {                               // a 2 x 2 block
        const double p = 0.5 * (y - x);
        const double q = p * p + w;
        double z = sqrt(fabs(q));
        x += shift;
        if (t == 0) {
          if (q >= 0.0) {
            z = p + ns_sgn(z, p);
            wr[nn - 1] = wr[nn] = x + z;
            if (z != 0.0) wr[nn] = x - w / z;
            wi[nn - 1] = wi[nn] = 0.0;
          } else {
            wr[nn - 1] = wr[nn] = x + p;
            wi[nn - 1] = z;
            wi[nn] = -z;
          }
        }
        nn -= 2;
        break;
      }
      if (its >= kNsQrMaxIts) {
        fail = 1;
        break;
      }
      if (ns_exceptional(its)) {                        // exceptional shift
        shift += x;
        for (int i = t; i <= nn; i += 64) HB(i, i) -= x;
        ns_wave_fence();
        const double s = ns_exceptional_top(its) ? fabs(HB(l + 1, l)) + fabs(HB(l + 2, l + 1))
                                                  : fabs(HB(nn, nn - 1)) + fabs(HB(nn - 1, nn - 2));
        x = y = 0.75 * s;
        w = -0.4375 * s * s;
      }
      ++its;
      // start of the double step: largest m in [l, nn-2] where two consecutive
      // sub-diagonals are small enough, m = l otherwise
      int m = l;
      for (int base = nn - 2; base >= l; base -= 64) {
        const int m0 = base - t;
        bool hit = m0 == l;
        if (m0 > l) {
          const double z0 = HB(m0, m0);
          double r0 = x - z0;
          const double s0 = y - z0;
          double p0 = (r0 * s0 - w) / HB(m0 + 1, m0) + HB(m0, m0 + 1);
          double q0 = HB(m0 + 1, m0 + 1) - z0 - r0 - s0;
          r0 = HB(m0 + 2, m0 + 1);
          const double ss = fabs(p0) + fabs(q0) + fabs(r0);
          p0 /= ss;
          q0 /= ss;
          r0 /= ss;
          const double u = fabs(HB(m0, m0 - 1)) * (fabs(q0) + fabs(r0));
          const double vv = fabs(p0) * (fabs(HB(m0 - 1, m0 - 1)) + fabs(z0) + fabs(HB(m0 + 1, m0 + 1)));
          hit = u <= kNsEps * vv;
        }
        const unsigned long long mask = __ballot(hit);
        if (mask) {
          m = base - (__ffsll(mask) - 1);
          break;
        }
      }
      double p, q, r;
      {
        const double z = HB(m, m);
        r = x - z;
        const double s0 = y - z;
        p = (r * s0 - w) / HB(m + 1, m) + HB(m, m + 1);
        q = HB(m + 1, m + 1) - z - r - s0;
        r = HB(m + 2, m + 1);
        const double s = fabs(p) + fabs(q) + fabs(r);
        p /= s;
        q /= s;
        r /= s;
      }
      for (int i = m + 2 + t; i <= nn; i += 64) {
        HB(i, i - 2) = 0.0;
        if (i != m + 2) HB(i, i - 3) = 0.0;
      }
      ns_wave_fence();
      // bulge chase over the active window [l, nn]; c[it]: column k-1 after the
      // previous step's column update, row l + t + 64 it
      double c[kNsQrIt];
#pragma unroll
      for (int it = 0; it < kNsQrIt; ++it) c[it] = 0.0;
#define NS_LANE(idx) ns_lane_value(c[0], c[1], c[2], (idx))
      for (int k = m; k <= nn - 1; ++k) {
        const bool notlast = (k != nn - 1);
        if (k != m) {
          p = NS_LANE(k - l);
          q = NS_LANE(k + 1 - l);
          r = notlast ? NS_LANE(k + 2 - l) : 0.0;
        }
        const NsHouse h = ns_house3(p, q, r);
        p = h.p;
        q = h.q;
        r = h.r;
        const double s = h.s;
        const int imax = (nn < k + 3) ? nn : k + 3;
        if (s == 0.0) {
          // no reflection at this step: the next one reads column k from
          // memory.  The loads are waited for here, on this rare path, so
          // that the loop head does not wait for all LDS operations.
#pragma unroll
          for (int it = 0; it < kNsQrIt; ++it) {
            const int i = l + t + 64 * it;
            if (i <= imax) c[it] = HB(i, k);
          }
          __builtin_amdgcn_s_waitcnt(kNsWaitLds);
          continue;
        }
        if (t == 0) {
          if (k == m) {
            if (l != m) HB(k, k - 1) = -HB(k, k - 1);
          } else {
            HB(k, k - 1) = ldexp(-s, h.e);
          }
        }
        const double pp = p + s;
        const double is = ns_recip(s), ipp = ns_recip(pp);
        const double x1 = pp * is, y1 = q * is, z1 = r * is;
        const double q1 = q * ipp, r1 = r * ipp;
        // rows k..k+2, columns k..nn.  Loads are unconditional at clamped,
        // valid addresses (a masked load would end its branch with a wait);
        // on the last step the third row is a copy of the second, weighted
        // by r1 = 0, and not stored.
        const int k2 = notlast ? k + 2 : k + 1;
        double a0[kNsQrIt], a1[kNsQrIt], a2[kNsQrIt];
#pragma unroll
        for (int it = 0; it < kNsQrIt; ++it) {
          const int j = min(k + t + 64 * it, nn);
          a0[it] = HB(k, j);
          a1[it] = HB(k + 1, j);
          a2[it] = HB(k2, j);
        }
#pragma unroll
        for (int it = 0; it < kNsQrIt; ++it) {
          const int j = k + t + 64 * it;
          double pv = a0[it] + q1 * a1[it];
          pv += r1 * a2[it];
          if (j <= nn) {
            if (notlast) HB(k + 2, j) = a2[it] - pv * z1;
            HB(k + 1, j) = a1[it] - pv * y1;
            HB(k, j) = a0[it] - pv * x1;
          }
        }
        ns_wave_fence();
        // columns k..k+2, rows l..min(nn, k+3), loaded the same way
#pragma unroll
        for (int it = 0; it < kNsQrIt; ++it) {
          const int i = min(l + t + 64 * it, imax);
          a0[it] = HB(i, k);
          a1[it] = HB(i, k + 1);
          a2[it] = HB(i, k2);
        }
#pragma unroll
        for (int it = 0; it < kNsQrIt; ++it) {
          const int i = l + t + 64 * it;
          double pv = x1 * a0[it] + y1 * a1[it];
          pv += z1 * a2[it];
          c[it] = a0[it] - pv;
          if (i <= imax) {
            if (notlast) HB(i, k + 2) = a2[it] - pv * r1;
            HB(i, k + 1) = a1[it] - pv * q1;
            HB(i, k) = c[it];
          }
        }
        ns_wave_fence();
      }
    }
  }
  ns_wave_fence();
#undef NS_LANE
#undef HB
  return fail;
}

constexpr int kNsMsFrom = 64;     // orders from which the multishift kernel below takes over

__global__ __launch_bounds__(64) void ns_qr_kernel(double* __restrict__ work, int n, int nv) {
  __shared__ double hb[ns_band_doubles(kNsMsFrom)];
  const NsWork ws = ns_work_split(work, n, nv);
  NsTeam<64> tm{nullptr};
  ns_band_fill(tm, ws.A, n, ws.hsub, n, hb, ws.HT);
  __syncthreads();
  const int fail = ns_qr_values_wave(hb, n, ws.wr0, ws.wi0, ws.misc);
  if (threadIdx.x == 0) ws.misc[1] = fail;
}

// ---- eigenvalue QR from order kNsMsFrom: multishift sweeps by one workgroup ----------------
// ns_ms_run (nonsym_core.hpp) with a team of one wave per bulge.  The band
// lives in LDS up to order kNsMsLds (with the sweep scratch, 162.2 KB of the
// 160 KiB).  Above that its columns below kNsMsLds are in LDS and the rest in
// the work buffer (NsSplitBand: accesses through generic pointers) until the
// deflations have shrunk the leading block to that order; from then on it is
// all in LDS.  Wave 0 computes each sweep's shifts with the one-wave loop
// above on the trailing block.
constexpr int kNsMsThreads = 64 * kNsMsBulges;
constexpr int kNsMsLds = 196;

struct NsWaveSmallEig {
  int* flag;
  __device__ int operator()(double* sb, int ns, double* sr, double* si, double tol) const {
    if (threadIdx.x < 64) {
      const int f = ns_qr_values_wave(sb, ns, sr, si, nullptr, tol);
      if (threadIdx.x == 0) *flag = f;
    }
    __syncthreads();
    return *flag;
  }
};

template <bool LDS>
__global__ __launch_bounds__(kNsMsThreads) void ns_qr_ms_kernel(double* __restrict__ work, int n, int nv) {
  __shared__ double band[ns_band_doubles(kNsMsLds)];
  __shared__ double scr[ns_ms_scratch_doubles()];
  __shared__ double red[kNsMsThreads / 64];
  __shared__ int flag;
  const NsWork ws = ns_work_split(work, n, nv);
  NsTeam<kNsMsThreads> tm{red};
  const NsWaveSmallEig small{&flag};
  int nn = n - 1, fail = 0;
  double shift = 0.0;
  if (LDS) {
    ns_band_fill(tm, ws.A, n, ws.hsub, n, band, ws.HT);
    __syncthreads();
    const double anorm = ns_band_norm(tm, NsBand{band}, n);
    fail = ns_ms_run(tm, NsBand{band}, nn, shift, anorm, -1, ws.wr0, ws.wi0, scr, small);
    if (threadIdx.x == 0) ws.misc[0] = anorm;
  } else {
    // columns below kNsMsLds in LDS, the rest in the work buffer, until the
    // deflations have shrunk the leading block to fit the LDS band
    ns_band_fill(tm, ws.A, n, ws.hsub, n, ws.HB, ws.HT);
    __syncthreads();
    const double anorm = ns_band_norm(tm, NsBand{ws.HB}, n);
    const int cnt = kNsMsLds * (kNsMsLds + 7) / 2;
    for (int e = threadIdx.x; e < cnt; e += kNsMsThreads) band[e] = ws.HB[e];
    __syncthreads();
    fail = ns_ms_run(tm, NsSplitBand{band, ws.HB, kNsMsLds}, nn, shift, anorm, kNsMsLds - 1, ws.wr0, ws.wi0, scr,
                     small);
    if (!fail) fail = ns_ms_run(tm, NsBand{band}, nn, shift, anorm, -1, ws.wr0, ws.wi0, scr, small);
    if (threadIdx.x == 0) ws.misc[0] = anorm;
  }
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
  if (n < kNsMsFrom)
    hipLaunchKernelGGL(ns_qr_kernel, dim3(1), dim3(64), 0, s, work, n, nv);
  else if (n <= kNsMsLds)
    hipLaunchKernelGGL(ns_qr_ms_kernel<true>, dim3(1), dim3(kNsMsThreads), 0, s, work, n, nv);
  else
    hipLaunchKernelGGL(ns_qr_ms_kernel<false>, dim3(1), dim3(kNsMsThreads), 0, s, work, n, nv);
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
