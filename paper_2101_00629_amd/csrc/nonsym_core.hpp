// Small dense non-symmetric eigensolve for the Rayleigh-Ritz step of the
// collocation method (the projected matrix of Z^-1 A, paper Sec. 3.2, is not
// symmetric).  Stages, each written once as plain C++ for the host (unit
// tests) and the device (nonsym.hip):
//   1. Householder reduction to upper Hessenberg form H = Q Hh Q^T by a team
//      of threads; reflector j is kept below the sub-diagonal of column j.
//   2. All eigenvalues of Hh by the Francis double-shift QR iteration
//      (Golub & Van Loan, Sec. 7.5) restricted to the active window, without
//      forming the Schur vectors; one wave, on a banded copy of Hh.
//   3. Ranking by descending real part; a complex pair stays together with
//      the positive imaginary part first.
//   4. Eigenvectors of Hh for the wanted (leading) eigenvalues only, by
//      inverse iteration with the pivoted Hessenberg LU of Hh - lambda I in
//      complex arithmetic, one team per cluster (each row operation split
//      over the team); eigenvalues closer than a gap form a cluster whose
//      vectors are orthogonalised against each other after every solve.
//   5. Back-transformation x <- Q x (the reflectors of stage 1).
//   6. Output: column c real (unit 2-norm) or, for a pair, columns c, c+1 the
//      real and imaginary parts of one eigenvector with |re|^2 + |im|^2 = 1.
#pragma once
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include "sym_core.hpp"

namespace ka {

constexpr double kNsEps = 2.220446049250313e-16;
// eigenvalues closer than this, relative to the largest modulus, form a cluster
constexpr double kNsClusterGap = 1e-8;

// ---- work layout -------------------------------------------------------------------------
// A    n*n      Hessenberg reduction, reflectors below the sub-diagonal
// hsub n        sub-diagonal of Hh;  beta n   reflector coefficients
// wr0, wi0 2n   eigenvalues in QR order;  rank n (as doubles), wr, wi 2n sorted
// misc 8        [0] norm of Hh, [1] QR status
// V    n*nv     wanted vectors, element i of output column c at V[i*nv + c]
// F    nv*(n*n + 4n)  per-entry LU planes and multipliers (contiguous per entry)
// HT   n*n      row-major copy of Hh (rows of B = Hh - lambda I for the LU)
// (nv: column capacity, at least the wanted count plus one for a pair that
// straddles it)
// HB   n*(n+7)/2 + 8  banded copy of Hh for the QR iteration
struct NsWork {
  double *A, *hsub, *beta, *wr0, *wi0, *rank, *wr, *wi, *misc, *V, *F, *HB, *HT;
  int nv;
};

KA_HD constexpr size_t ns_band_doubles(int n) { return (size_t)n * (n + 7) / 2 + 8; }
KA_HD inline size_t ns_lu_doubles(int n) { return (size_t)n * n + 4 * (size_t)n; }

KA_HD inline size_t nonsym_work_doubles(int n, int nv) {
  return (size_t)2 * n * n + 8 * (size_t)n + 8 + (size_t)n * nv + (size_t)nv * ns_lu_doubles(n) + ns_band_doubles(n);
}

KA_HD inline NsWork ns_work_split(double* w, int n, int nv) {
  NsWork s;
  s.nv = nv;
  s.A = w;
  s.hsub = w + (size_t)n * n;
  s.beta = s.hsub + n;
  s.wr0 = s.beta + n;
  s.wi0 = s.wr0 + n;
  s.rank = s.wi0 + n;
  s.wr = s.rank + n;
  s.wi = s.wr + n;
  s.misc = s.wi + n;
  s.V = s.misc + 8;
  s.F = s.V + (size_t)n * nv;
  s.HB = s.F + (size_t)nv * ns_lu_doubles(n);
  s.HT = s.HB + ns_band_doubles(n);
  return s;
}

KA_HD inline double ns_sgn(double a, double b) { return b >= 0.0 ? fabs(a) : -fabs(a); }
KA_HD inline double ns_cabs(double a, double b) { return sqrt(a * a + b * b); }

// reciprocal for the reflector coefficients: two Newton steps on the
// hardware estimate on the device, a division on the host
KA_HD inline double ns_recip(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
#else
  return 1.0 / x;
#endif
}

// square root of x in [1/16, 4] (no scaling or special cases needed there):
// on the device the hardware reciprocal square root estimate refined by the
// coupled Newton iteration for sqrt(x) and 1/(2 sqrt(x)) (Markstein), one
// step for both and two more for the root; a library call on the host
KA_HD inline double ns_sqrt_mid(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  g = fma(fma(-g, g, x), h, g);
  return fma(fma(-g, g, x), h, g);
#else
  return sqrt(x);
#endif
}

// The 3 x 3 Householder data of a double-shift step from the vector
// (v0, v1, v2): the vector scaled by the power of two 2^-e that brings its
// largest magnitude into [1/2, 1) (exact; the reflection does not depend on
// the scale), s = +-||(p, q, r)|| with the sign of p (0 if the vector is
// zero), and e, so that the reflection leaves -s 2^e in the first entry.
struct NsHouse {
  double p, q, r, s;
  int e;
};
KA_HD inline NsHouse ns_house3(double v0, double v1, double v2) {
  const double m = fmax(fmax(fabs(v0), fabs(v1)), fabs(v2));
  NsHouse h{0.0, 0.0, 0.0, 0.0, 0};
  if (m == 0.0) return h;
#ifdef __HIP_DEVICE_COMPILE__
  h.e = __builtin_amdgcn_frexp_exp(m);
#else
  frexp(m, &h.e);
#endif
  h.p = ldexp(v0, -h.e);
  h.q = ldexp(v1, -h.e);
  h.r = ldexp(v2, -h.e);
  h.s = ns_sgn(ns_sqrt_mid(h.p * h.p + h.q * h.q + h.r * h.r), h.p);
  return h;
}

// ---- stage 1: Hessenberg reduction by a team ---------------------------------------------
// A: n x n with leading dimension ld (fast memory if available).  v, w: team
// scratch of >= n doubles each.  Team interface as in sym_core.hpp.
// loads per thread that the Hessenberg reduction issues together: 8 where A
// lives in device memory, 2 where it is in LDS (there more only costs
// registers)
template <int kNsBatch = 8, class Team>
KA_HD void ns_hessenberg(Team& tm, double* A, int ld, int n, double* hsub, double* beta, double* v, double* w) {
  const int t = tm.tid(), NT = tm.size();
#define AH(i, j) A[(i) + (size_t)(j) * ld]
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    double ss = 0.0;
    for (int i = t; i < m; i += NT) ss += AH(j + 1 + i, j) * AH(j + 1 + i, j);
    ss = tm.sum(ss);
    const double x0 = AH(j + 1, j);
    const double alpha = -ns_sgn(sqrt(ss), x0);
    const double v0 = x0 - alpha;
    const bool skip = !(ss > 1e-300);
    const double b = skip ? 0.0 : 2.0 / (ss - x0 * x0 + v0 * v0);
    for (int i = t; i < m; i += NT) v[i] = (i == 0) ? v0 : AH(j + 1 + i, j);
    if (t == 0) {
      hsub[j] = skip ? x0 : alpha;
      beta[j] = b;
    }
    tm.sync();
    if (!skip) {
      // Each loop below issues kNsBatch loads per thread together, so that
      // enough are in flight when A lives in device memory; the dot products
      // keep eight partial sums added in a fixed tree.
      // left: A[j+1:, c] -= b v (v^T A[j+1:, c]) for c > j (a thread per column)
      for (int c = j + 1 + t; c < n; c += NT) {
        const double* col = &AH(j + 1, c);
        double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int i = 0;
        for (; i + kNsBatch - 1 < m; i += kNsBatch) {
          double a[kNsBatch];
#pragma unroll
          for (int u = 0; u < kNsBatch; ++u) a[u] = col[i + u];
#pragma unroll
          for (int u = 0; u < kNsBatch; ++u) acc[u % 8] += v[i + u] * a[u];
        }
        for (; i < m; ++i) acc[0] += v[i] * col[i];
        w[c] = b * (((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7])));
      }
      tm.sync();
      // the rank-one updates: thread t takes row t % (rows) in the columns of
      // its group t / (rows), so that consecutive threads touch consecutive
      // rows (each element takes the same single update as in a row-by-row loop)
      {
        const int nc = n - j - 1, groups = NT >= m ? NT / m : 1;
        for (int r0 = t; r0 < (NT >= m ? groups * m : m); r0 += NT) {
          const int i = NT >= m ? r0 % m : r0, g = NT >= m ? r0 / m : 0;
          double* row = &AH(j + 1 + i, j + 1);
          const double vi = v[i];
          int c = g;
          for (; c + (kNsBatch - 1) * groups < nc; c += kNsBatch * groups) {
            double a[kNsBatch];
#pragma unroll
            for (int u = 0; u < kNsBatch; ++u) a[u] = row[(size_t)(c + u * groups) * ld];
#pragma unroll
            for (int u = 0; u < kNsBatch; ++u) row[(size_t)(c + u * groups) * ld] = a[u] - w[j + 1 + c + u * groups] * vi;
          }
          for (; c < nc; c += groups) row[(size_t)c * ld] -= w[j + 1 + c] * vi;
        }
      }
      tm.sync();
      // right: A[r, j+1:] -= b (A[r, j+1:] v) v^T for every row (a thread per row)
      for (int r = t; r < n; r += NT) {
        const double* row = &AH(r, j + 1);
        double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int i = 0;
        for (; i + kNsBatch - 1 < m; i += kNsBatch) {
          double a[kNsBatch];
#pragma unroll
          for (int u = 0; u < kNsBatch; ++u) a[u] = row[(size_t)(i + u) * ld];
#pragma unroll
          for (int u = 0; u < kNsBatch; ++u) acc[u % 8] += a[u] * v[i + u];
        }
        for (; i < m; ++i) acc[0] += row[(size_t)i * ld] * v[i];
        w[r] = b * (((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7])));
      }
      tm.sync();
      {
        const int groups = NT >= n ? NT / n : 1;
        for (int r0 = t; r0 < (NT >= n ? groups * n : n); r0 += NT) {
          const int r = NT >= n ? r0 % n : r0, g = NT >= n ? r0 / n : 0;
          double* row = &AH(r, j + 1);
          const double wr = w[r];
          int i = g;
          for (; i + (kNsBatch - 1) * groups < m; i += kNsBatch * groups) {
            double a[kNsBatch];
#pragma unroll
            for (int u = 0; u < kNsBatch; ++u) a[u] = row[(size_t)(i + u * groups) * ld];
#pragma unroll
            for (int u = 0; u < kNsBatch; ++u) row[(size_t)(i + u * groups) * ld] = a[u] - wr * v[i + u * groups];
          }
          for (; i < m; i += groups) row[(size_t)i * ld] -= wr * v[i];
        }
      }
    }
    tm.sync();
    for (int i = t; i < m; i += NT) AH(j + 1 + i, j) = v[i];   // reflector
    tm.sync();
  }
  if (t == 0 && n >= 2) hsub[n - 2] = AH(n - 1, n - 2);
  tm.sync();
#undef AH
}

// ---- stage 2: eigenvalues of Hh (double-shift QR, no Schur vectors) -----------------------
// hb: banded column storage, element (i, j) for i <= j + 3 at hb[j (j + 7) / 2 + i]
// (the sub-diagonal, the two bulge diagonals and the upper triangle).
KA_HD inline size_t ns_band_index(int i, int j) { return (size_t)j * (j + 7) / 2 + i; }

// Band storage as the QR stages see it: entry (i, j) at col(j)[i].  NsBand is
// one array; NsSplitBand keeps the columns below `cut` in one array (LDS on
// the device) and the rest in another (device memory), both at the packed
// index above, so the columns below `cut` need no copy when the band moves
// wholly into the first array.  Columns below contig() are in the first
// array, the others in the second (kSplit: whether there is a second);
// first_col(j) and second_col(j) give a column's storage as a pointer derived
// from that array alone, so that code using only such pointers is compiled for
// that array's address space.
struct NsBand {
  static constexpr bool kSplit = false;
  double* p;
  KA_HD double* col(int j) const { return p + ns_band_index(0, j); }
  KA_HD int contig() const { return 1 << 30; }
  KA_HD double* first_col(int j) const { return p + ns_band_index(0, j); }
  KA_HD double* second_col(int j) const { return p + ns_band_index(0, j); }
};
struct NsSplitBand {
  static constexpr bool kSplit = true;
  double* lo;
  double* hi;
  int cut;
  KA_HD double* col(int j) const { return (j < cut ? lo : hi) + ns_band_index(0, j); }
  KA_HD int contig() const { return cut; }
  KA_HD double* first_col(int j) const { return lo + ns_band_index(0, j); }
  KA_HD double* second_col(int j) const { return hi + ns_band_index(0, j); }
};

// Fill the banded copy (and, if given, the row-major copy HT) from stage 1's
// output (team, then sync by the caller).
template <class Team>
KA_HD void ns_band_fill(Team& tm, const double* A, int ld, const double* hsub, int n, double* hb, double* HT) {
  const int t = tm.tid(), NT = tm.size();
  for (int j = 0; j < n; ++j)
    for (int i = t; i <= j + 3; i += NT) {
      double x = 0.0;
      if (i <= j) x = A[i + (size_t)j * ld];
      else if (i == j + 1 && i < n) x = hsub[j];
      hb[ns_band_index(i, j)] = x;
    }
  if (HT)
    for (int i = 0; i < n; ++i)
      for (int j = t; j < n; j += NT) HT[(size_t)i * n + j] = (j >= i) ? A[i + (size_t)j * ld] : (j == i - 1 ? hsub[j] : 0.0);
}

// Scalar control flow is identical in every thread (all read the same values
// after a barrier); row and column updates are split over the team.
// Returns 0, or 1 when an eigenvalue needed more than 60 iterations.
// Iteration control of the double-shift QR, per deflation: exceptional
// shifts after 10 and 20 iterations and then after every further 10, from 30
// on alternating between the sub-diagonals at the bottom and at the top of
// the active window, so that a window that stalls under one shift gets a
// different one; the iteration gives up after kNsQrMaxIts.
constexpr int kNsQrMaxIts = 200;
KA_HD inline bool ns_exceptional(int its) { return its > 0 && its % 10 == 0; }
KA_HD inline bool ns_exceptional_top(int its) { return its >= 30 && (its / 10) % 2 == 1; }

// One Francis double step on the active window [l, nn] (no negligible
// sub-diagonal inside it).  (x, y, w) describe the shifts: x and y the
// trailing diagonal entries and w the product of the trailing off-diagonal
// pair, or the exceptional values.  The step starts at the largest m in
// [l, nn-2] below which two consecutive sub-diagonal entries are small
// enough, else at l, and chases one 3x3 bulge to the bottom.
template <class Team, class Band>
KA_HD void ns_ds_iteration(Team& tm, const Band& B, int l, int nn, double x, double y, double w) {
  const int t = tm.tid(), NT = tm.size();
#define HB(i, j) (B.col(j)[i])
  int m;
  double p = 0.0, q = 0.0, r = 0.0, z = 0.0;
  for (m = nn - 2; m >= l; --m) {
    z = HB(m, m);
    r = x - z;
    const double s0 = y - z;
    p = (r * s0 - w) / HB(m + 1, m) + HB(m, m + 1);
    q = HB(m + 1, m + 1) - z - r - s0;
    r = HB(m + 2, m + 1);
    const double s = fabs(p) + fabs(q) + fabs(r);
    p /= s;
    q /= s;
    r /= s;
    if (m == l) break;
    const double u = fabs(HB(m, m - 1)) * (fabs(q) + fabs(r));
    const double vv = fabs(p) * (fabs(HB(m - 1, m - 1)) + fabs(z) + fabs(HB(m + 1, m + 1)));
    if (u <= kNsEps * vv) break;
  }
  tm.sync();
  for (int i = m + 2 + t; i <= nn; i += NT) {
    HB(i, i - 2) = 0.0;
    if (i != m + 2) HB(i, i - 3) = 0.0;
  }
  tm.sync();
  // bulge chase over the active window [l, nn]
  for (int k = m; k <= nn - 1; ++k) {
    const bool notlast = (k != nn - 1);
    if (k != m) {
      p = HB(k, k - 1);
      q = HB(k + 1, k - 1);
      r = notlast ? HB(k + 2, k - 1) : 0.0;
    }
    const NsHouse h = ns_house3(p, q, r);
    p = h.p;
    q = h.q;
    r = h.r;
    const double s = h.s;
    tm.sync();
    if (s == 0.0) continue;
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
    for (int j = k + t; j <= nn; j += NT) {
      double pv = HB(k, j) + q1 * HB(k + 1, j);
      if (notlast) {
        pv += r1 * HB(k + 2, j);
        HB(k + 2, j) -= pv * z1;
      }
      HB(k + 1, j) -= pv * y1;
      HB(k, j) -= pv * x1;
    }
    tm.sync();
    const int imax = (nn < k + 3) ? nn : k + 3;
    for (int i = l + t; i <= imax; i += NT) {
      double pv = x1 * HB(i, k) + y1 * HB(i, k + 1);
      if (notlast) {
        pv += z1 * HB(i, k + 2);
        HB(i, k + 2) -= pv * r1;
      }
      HB(i, k + 1) -= pv * q1;
      HB(i, k) -= pv;
    }
    tm.sync();
  }
#undef HB
}

// Deflation of the bottom of the active window: one real eigenvalue (l == nn)
// or the two eigenvalues of the trailing 2 x 2 block (l == nn - 1), written
// by thread 0 with the accumulated exceptional shift added back.
KA_HD inline void ns_deflate_2x2(double x, double y, double w, double shift, double* wr, double* wi, int nn) {
  const double p = 0.5 * (y - x);
  const double q = p * p + w;
  double z = sqrt(fabs(q));
  x += shift;
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

// tol: relative size of a negligible sub-diagonal entry (kNsEps for
// eigenvalues; kNsShiftTol where they only serve as shifts)
template <class Team>
KA_HD int ns_qr_values(Team& tm, double* hb, int n, double* wr, double* wi, double* anorm_out, double tol = kNsEps) {
  const int t = tm.tid(), NT = tm.size();
#define HB(i, j) hb[ns_band_index((i), (j))]
  double anorm = 0.0;
  for (int j = t; j < n; j += NT)
    for (int i = 0; i <= j + 1 && i < n; ++i) anorm += fabs(HB(i, j));
  anorm = tm.sum(anorm);
  if (anorm_out && t == 0) *anorm_out = anorm;
  int nn = n - 1;
  double shift = 0.0;
  int fail = 0;
  while (nn >= 0 && !fail) {
    int its = 0;
    while (true) {
      tm.sync();
      int l;
      for (l = nn; l >= 1; --l) {
        double s = fabs(HB(l - 1, l - 1)) + fabs(HB(l, l));
        if (s == 0.0) s = anorm;
        if (fabs(HB(l, l - 1)) <= tol * s) break;
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
        if (t == 0) ns_deflate_2x2(x, y, w, shift, wr, wi, nn);
        nn -= 2;
        break;
      }
      if (its >= kNsQrMaxIts) {
        fail = 1;
        break;
      }
      if (ns_exceptional(its)) {                        // exceptional shift
        shift += x;
        tm.sync();
        for (int i = t; i <= nn; i += NT) HB(i, i) -= x;
        tm.sync();
        const double s = ns_exceptional_top(its) ? fabs(HB(l + 1, l)) + fabs(HB(l + 2, l + 1))
                                                  : fabs(HB(nn, nn - 1)) + fabs(HB(nn - 1, nn - 2));
        x = y = 0.75 * s;
        w = -0.4375 * s * s;
      }
      ++its;
      ns_ds_iteration(tm, NsBand{hb}, l, nn, x, y, w);
    }
  }
  tm.sync();
#undef HB
  return fail;
}

// ---- stage 2, large windows: multishift QR with a chain of small bulges ---------------
// For an active window of kNsMsMinWindow or more rows, one sweep applies ns
// shifts at once: the eigenvalues of the trailing ns x ns block, taken in
// pairs (a complex-conjugate pair or two real shifts), each pair driving
// one 3 x 3 bulge.  The bulges enter at the top of the window one after the
// other, three rows apart, and move down one row per round.  Within a round
// every bulge's reflector comes from the matrix as the previous round left
// it, then all row updates run, then all column updates.  Bulges three rows
// apart touch disjoint rows in the row phase and disjoint columns in the
// column phase.  Where one bulge's row update and another's column update
// overlap, they are a left and a right multiplication, which commute.  So a
// round is a reordering of applying the bulges one at a time, bottom first,
// and the team applies each phase in parallel.  The entries a reflector
// annihilates are stored as zeros, because the bulge behind passes over them.
// Deflation and exceptional shifts are handled as in ns_qr_values (same
// checks, double steps); a window below kNsMsMinWindow goes to the small
// solver whole.
constexpr int kNsMsMax = 16;          // most shifts per sweep
// The trailing block's eigenvalues only steer a sweep, so its QR stops at
// this relative sub-diagonal size.  On the Rayleigh-Ritz matrices of the
// collocation solves (orders 114 to 228) 1e-4 takes 4% less time than 1e-8
// over all QR calls (the small QR of the shifts runs on one wave while the
// others wait); dense random test matrices take about 15% longer on the host.
// The eigenvalues themselves deflate at machine precision either way.
constexpr double kNsShiftTol = 1e-4;
constexpr int kNsMsMinWindow = 24;    // smaller windows go to the small solver
KA_HD inline int ns_ms_shifts(int win) {
  const int s = win >= 96 ? kNsMsMax : (win / 6) & ~1;
  return s < 4 ? 4 : s;
}
constexpr int kNsMsBulges = kNsMsMax / 2;
// team-shared scratch of the multishift driver: the trailing block (band
// layout), the shifts, and two reflector tables (this round's and the next
// round's) of 8 doubles per bulge
// sweep scratch: the small solver's band, the shifts, the reflector tables,
// and the eigenvalues of a small window (at the end, past the band of a
// window below kNsMsMinWindow, which overlays the shifts and tables)
KA_HD constexpr size_t ns_ms_window_values() {
  return ns_band_doubles(kNsMsMax) + 2 * kNsMsMax + 2 * 8 * kNsMsBulges + 8;
}
KA_HD constexpr size_t ns_ms_scratch_doubles() { return ns_ms_window_values() + 2 * kNsMsMinWindow; }
static_assert(ns_band_doubles(kNsMsMinWindow - 1) <= ns_ms_window_values(),
              "the band of a small window fits before its eigenvalues");

// largest l in [1, nn] with a negligible sub-diagonal H(l, l-1), else 0
// (each thread scans its own positions from the top, then a team maximum)
template <class Team, class Band>
KA_HD int ns_find_split(Team& tm, const Band& B, int nn, double anorm) {
  const int t = tm.tid(), NT = tm.size();
  int best = 0;
  for (int l0 = nn - t; l0 >= 1; l0 -= NT) {
    double s = fabs(B.col(l0 - 1)[l0 - 1]) + fabs(B.col(l0)[l0]);
    if (s == 0.0) s = anorm;
    if (fabs(B.col(l0 - 1)[l0]) <= kNsEps * s) {
      best = l0;
      break;
    }
  }
  return tm.imax(best);
}

// Reorder ns shifts (conjugate pairs adjacent, positive imaginary part first,
// as ns_qr_values leaves them) so that entries 2b, 2b+1 form the pair of
// bulge b: the complex pairs first, then the real shifts in descending order
// taken two at a time.  ns is even, so the real shifts are even in number.
KA_HD inline void ns_pair_shifts(double* sr, double* si, int ns) {
  double tr[kNsMsMax], ti[kNsMsMax];
  int o = 0;
  for (int i = 0; i < ns; ++i)
    if (si[i] != 0.0) {
      tr[o] = sr[i];
      ti[o++] = si[i];
    }
  const int nc = o;
  for (int i = 0; i < ns; ++i)
    if (si[i] == 0.0) {
      int j = o++;
      for (; j > nc && tr[j - 1] < sr[i]; --j) tr[j] = tr[j - 1];
      tr[j] = sr[i];
    }
  for (int i = nc; i < ns; ++i) ti[i] = 0.0;
  for (int i = 0; i < ns; ++i) {
    sr[i] = tr[i];
    si[i] = ti[i];
  }
}

// First column of (H - s1 I)(H - s2 I) at the top of the window, rows l..l+2,
// up to a positive factor (divided by |h00 - s2| + |Im s2| + |h10| against
// overflow); s1, s2 both real or a conjugate pair.
template <class Band>
KA_HD inline void ns_ms_first_column(const Band& B, int l, double sr1, double si1, double sr2, double si2,
                                     double* v) {
  const double h00 = B.col(l)[l], h10 = B.col(l)[l + 1];
  const double h01 = B.col(l + 1)[l], h11 = B.col(l + 1)[l + 1];
  const double h21 = B.col(l + 1)[l + 2];
  const double s = fabs(h00 - sr2) + fabs(si2) + fabs(h10);
  if (s == 0.0) {
    v[0] = v[1] = v[2] = 0.0;
    return;
  }
  const double h10s = h10 / s;
  v[0] = h10s * h01 + (h00 - sr1) * ((h00 - sr2) / s) - si1 * (si2 / s);
  v[1] = h10s * (h00 + h11 - sr1 - sr2);
  v[2] = h10s * h21;
}

// Reflector of a bulge at step k from v = the entries (k..k+2, k-1), or at
// k = l from the shift polynomial's first column: R[0] = 1 if there is a
// reflection, R[1..5] = the coefficients of the row and column updates.  For
// k > l the column k-1 is set to what the reflection leaves (-s 2^e, 0, 0).
// (computed by every thread of a group from the same values; only the one
// with store set writes the matrix and the table entry R)
struct NsRefl {
  double f, x1, y1, z1, q1, r1;   // f = 1 if there is a reflection
};
template <class Band>
KA_HD inline NsRefl ns_ms_reflector_g(const Band& B, int l, int nn, int k, double v0, double v1, double v2, double* R,
                                      bool store) {
  const bool notlast = k != nn - 1;
  if (!notlast) v2 = 0.0;
  NsRefl c{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const NsHouse h = ns_house3(v0, v1, v2);
  if (h.s == 0.0) {
    if (store) R[0] = 0.0;
    return c;
  }
  const double pp = h.p + h.s;
  const double is = ns_recip(h.s), ipp = ns_recip(pp);
  c = NsRefl{1.0, pp * is, h.q * is, h.r * is, h.q * ipp, h.r * ipp};
  if (store) {
    if (k > l) {
      const double sub = ldexp(-h.s, h.e);
      auto put = [&](double* c) {
        c[k] = sub;
        c[k + 1] = 0.0;
        if (notlast) c[k + 2] = 0.0;
      };
      if (!Band::kSplit || k - 1 < B.contig())
        put(B.first_col(k - 1));
      else
        put(B.second_col(k - 1));
    }
    R[0] = c.f;
    R[1] = c.x1;
    R[2] = c.y1;
    R[3] = c.z1;
    R[4] = c.q1;
    R[5] = c.r1;
  }
  return c;
}

// One multishift sweep over the window [l, nn] with nb bulges (shift pairs
// sr/si[2b], [2b+1]).  rt: team-shared, two tables of 8 doubles per bulge
// (this round's reflectors and the next round's).  Bulge b takes steps
// k = l .. nn-1 in rounds 3b .. 3b + nn-1-l.  The team works in groups of
// tm.gsize() threads (a wave on the device, one thread on the host), group g
// taking bulges g, g + groups, ...  A round is two phases, with a team
// barrier after each:
//  - rows: each bulge's rows k..k+2 over columns k..nn;
//  - columns: each bulge's columns k..k+2 over rows l..min(nn, k+3); then
//    the group forms the bulge's next reflector from the entries
//    (k+1..k+3, k) it has just computed, picked from the threads that hold
//    them (every thread of the group computes it, the first one stores it).
// A group's threads run over consecutive columns (rows phase) or rows
// (columns phase), four at a time with the loads first.  On the last step
// (k = nn-1) the third row or column is a copy of the second with weight 0
// (the reflector has r = 0), so that the arithmetic has no branch and every
// load is issued with the others; only its store is skipped.  A group with a
// single bulge (every group on the device) keeps its coefficients in
// registers; otherwise they come from the table.
template <class Team, class Band>
KA_HD void ns_ms_sweep(Team& tm, const Band& B, int l, int nn, const double* sr, const double* si, int nb, double* rt) {
  const int t = tm.tid(), NT = tm.size(), G = tm.gsize();
  const int grp = tm.group(), lane = t - grp * G, ngrp = NT / G;
  const bool own = ngrp >= nb;
#define HB(i, j) (B.col(j)[i])
  for (int i = l + 2 + t; i <= nn; i += NT) {
    HB(i, i - 2) = 0.0;
    if (i >= l + 3) HB(i, i - 3) = 0.0;
  }
  tm.sync();
  NsRefl mine{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};           // this round's reflector of the group's bulge (own)
  if (grp == 0) {
    double v[3];
    ns_ms_first_column(B, l, sr[0], si[0], sr[1], si[1], v);
    tm.gsync();
    mine = ns_ms_reflector_g(B, l, nn, l, v[0], v[1], v[2], rt, lane == 0);
  }
  const int rounds = 3 * (nb - 1) + (nn - l);
  for (int rd = 0; rd < rounds; ++rd) {
    tm.sync();
    const double* R = rt + (rd & 1) * 8 * kNsMsBulges;
    double* Rn = rt + ((rd + 1) & 1) * 8 * kNsMsBulges;
    for (int b = grp; b < nb; b += ngrp) {             // rows phase
      const int k = l + rd - 3 * b;
      if (k < l || k > nn - 1) continue;
      const NsRefl c = own ? mine : NsRefl{R[8 * b], R[8 * b + 1], R[8 * b + 2], R[8 * b + 3], R[8 * b + 4], R[8 * b + 5]};
      if (c.f == 0.0) continue;
      const bool notlast = k != nn - 1;
      const int k2 = notlast ? k + 2 : k + 1;
      auto rowupd = [&](int ja, int jb, auto colf) {   // columns ja..jb, all in one array
        for (int j0 = ja + lane; j0 <= jb; j0 += 4 * G) {
          double a0[4], a1[4], a2[4];
          double* col[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int j = j0 + u * G <= jb ? j0 + u * G : jb;
            col[u] = colf(j);
            a0[u] = col[u][k];
            a1[u] = col[u][k + 1];
            a2[u] = col[u][k2];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double pv = a0[u] + c.q1 * a1[u] + c.r1 * a2[u];   // r1 = 0 on the last step
            if (j0 + u * G <= jb) {
              if (notlast) col[u][k + 2] = a2[u] - pv * c.z1;
              col[u][k + 1] = a1[u] - pv * c.y1;
              col[u][k] = a0[u] - pv * c.x1;
            }
          }
        }
      };
      if constexpr (Band::kSplit) {
        // the first G columns in the second array are loaded before the
        // columns in the first, so that their (longer) latency overlaps
        const int cut = B.contig(), ga = k > cut ? k : cut;
        const bool hasg = nn >= ga;
        double g0 = 0.0, g1 = 0.0, g2 = 0.0;
        double* gc = nullptr;
        if (hasg) {
          gc = B.second_col(ga + lane <= nn ? ga + lane : nn);
          g0 = gc[k];
          g1 = gc[k + 1];
          g2 = gc[k2];
        }
        if (k < cut) rowupd(k, nn < cut ? nn : cut - 1, [&](int j) { return B.first_col(j); });
        if (hasg) {
          if (ga + lane <= nn) {
            const double pv = g0 + c.q1 * g1 + c.r1 * g2;
            if (notlast) gc[k + 2] = g2 - pv * c.z1;
            gc[k + 1] = g1 - pv * c.y1;
            gc[k] = g0 - pv * c.x1;
          }
          if (nn >= ga + G) rowupd(ga + G, nn, [&](int j) { return B.second_col(j); });
        }
      } else {
        rowupd(k, nn, [&](int j) { return B.col(j); });
      }
    }
    tm.sync();
    for (int b = grp; b < nb; b += ngrp) {             // columns phase, then the next reflector
      const int k = l + rd - 3 * b, kn = k + 1;
      const NsRefl c = own ? mine : NsRefl{R[8 * b], R[8 * b + 1], R[8 * b + 2], R[8 * b + 3], R[8 * b + 4], R[8 * b + 5]};
      const bool upd = k >= l && k <= nn - 1 && c.f != 0.0;
      double keep0 = 0.0, keep1 = 0.0, keep2 = 0.0;   // new (k+1..k+3, k) in the threads that computed them
      if (upd) {
        const bool notlast = k != nn - 1;
        const int imax = nn < k + 3 ? nn : k + 3;
        const int k2 = notlast ? k + 2 : k + 1;
        auto colupd = [&](double* c0, double* c1, double* c2) {   // the three columns (uniform in a group)
          for (int i0 = l + lane; i0 <= imax; i0 += 4 * G) {
            double a0[4], a1[4], a2[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = i0 + u * G <= imax ? i0 + u * G : imax;
              a0[u] = c0[i];
              a1[u] = c1[i];
              a2[u] = c2[i];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = i0 + u * G;
              const double pv = c.x1 * a0[u] + c.y1 * a1[u] + c.z1 * a2[u];   // z1 = 0 on the last step
              if (i <= imax) {
                if (notlast) c2[i] = a2[u] - pv * c.r1;
                c1[i] = a1[u] - pv * c.q1;
                const double h = a0[u] - pv;
                c0[i] = h;
                keep0 = i == k + 1 ? h : keep0;
                keep1 = i == k + 2 ? h : keep1;
                keep2 = i == k + 3 ? h : keep2;
              }
            }
          }
        };
        if (!Band::kSplit || k2 < B.contig())
          colupd(B.first_col(k), B.first_col(k + 1), B.first_col(k2));
        else if (k >= B.contig())
          colupd(B.second_col(k), B.second_col(k + 1), B.second_col(k2));
        else
          colupd(B.col(k), B.col(k + 1), B.col(k2));
      }
      NsRefl next{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (kn >= l && kn <= nn - 1) {
        if (upd) {                                     // (kn > l) from registers: no wait for the stores above
          const double v0 = tm.gpick(keep0, (k + 1 - l) % G);
          const double v1 = tm.gpick(keep1, (k + 2 - l) % G);
          const double v2 = k + 3 <= nn ? tm.gpick(keep2, (k + 3 - l) % G) : 0.0;
          next = ns_ms_reflector_g(B, l, nn, kn, v0, v1, v2, Rn + 8 * b, lane == 0);
        } else {
          double v[3];
          if (kn == l) {
            ns_ms_first_column(B, l, sr[2 * b], si[2 * b], sr[2 * b + 1], si[2 * b + 1], v);
          } else {                                     // no reflection this round: as the matrix holds them
            v[0] = HB(kn, kn - 1);
            v[1] = HB(kn + 1, kn - 1);
            v[2] = kn + 2 <= nn ? HB(kn + 2, kn - 1) : 0.0;
          }
          tm.gsync();                                  // every thread has read before the first one stores
          next = ns_ms_reflector_g(B, l, nn, kn, v[0], v[1], v[2], Rn + 8 * b, lane == 0);
        }
      } else if (lane == 0) {
        Rn[8 * b] = 0.0;
      }
      if (own) mine = next;
    }
  }
  tm.sync();
#undef HB
}

// All eigenvalues by multishift sweeps on large windows and the small solver
// on small ones (on a copy; a window [l, nn] split off by a negligible
// H(l, l-1) has eigenvalues of its own), for the leading block [0, nn] of the
// band B, until that block is below order stop + 1 (stop = -1: to the end).  nn and shift (the
// accumulated exceptional shift) carry the state between calls, so that a
// caller can move the band to faster storage between two calls.  anorm: the
// norm of the whole matrix.  scr: team-shared scratch of
// ns_ms_scratch_doubles().  small_eig(sb, ns, sr, si, tol): all eigenvalues
// of a band of order ns (copied to sb = scr: a window's trailing block for a
// sweep's shifts, with tol = kNsShiftTol, or a whole window below order
// kNsMsMinWindow, with tol = kNsEps), called by every thread,
// returning the same status to all.  Returns 0, or 1 when an
// eigenvalue needed more than kNsQrMaxIts iterations.  Inlined, so that each
// call site accesses its storage with the instructions of its address space.
template <class Team, class Band, class SmallEig>
KA_HD KA_FORCEINLINE int ns_ms_run(Team& tm, const Band& B, int& nn, double& shift, double anorm, int stop, double* wr,
                                   double* wi, double* scr, const SmallEig& small_eig) {
  const int t = tm.tid(), NT = tm.size();
  double* sb = scr;
  double* sr = sb + ns_band_doubles(kNsMsMax);
  double* si = sr + kNsMsMax;
  double* rt = si + kNsMsMax;
  double* wv = scr + ns_ms_window_values();
  int fail = 0;
#define HB(i, j) (B.col(j)[i])
  while (nn > stop && !fail) {
    int its = 0;
    while (true) {
      tm.sync();
      const int l = ns_find_split(tm, B, nn, anorm);
      double x = HB(nn, nn);
      if (l == nn) {
        if (t == 0) {
          wr[nn] = x + shift;
          wi[nn] = 0.0;
        }
        --nn;
        break;
      }
      double y = HB(nn - 1, nn - 1);
      double w = HB(nn, nn - 1) * HB(nn - 1, nn);
      if (l == nn - 1) {
        if (t == 0) ns_deflate_2x2(x, y, w, shift, wr, wi, nn);
        nn -= 2;
        break;
      }
      if (its >= kNsQrMaxIts) {
        fail = 1;
        break;
      }
      const bool ex = ns_exceptional(its);
      if (ex) {
        shift += x;
        tm.sync();
        for (int i = t; i <= nn; i += NT) HB(i, i) -= x;
        tm.sync();
        const double s = ns_exceptional_top(its) ? fabs(HB(l + 1, l)) + fabs(HB(l + 2, l + 1))
                                                  : fabs(HB(nn, nn - 1)) + fabs(HB(nn - 1, nn - 2));
        x = y = 0.75 * s;
        w = -0.4375 * s * s;
      }
      ++its;
      const int win = nn - l + 1;
      if (ex) {
        ns_ds_iteration(tm, B, l, nn, x, y, w);
        continue;
      }
      // one call of the small solver on a copy: a small window whole (its
      // eigenvalues are final), else the window's trailing block for the
      // sweep's shifts
      const bool whole = win < kNsMsMinWindow;
      const int ns = whole ? win : ns_ms_shifts(win), o = nn - ns + 1;
      for (int j = 0; j < ns; ++j)
        for (int i = t; i <= j + 3; i += NT) sb[ns_band_index(i, j)] = (i <= j + 1 && i < ns) ? HB(o + i, o + j) : 0.0;
      tm.sync();
      const int sf = small_eig(sb, ns, whole ? wv : sr, whole ? wv + kNsMsMinWindow : si, whole ? kNsEps : kNsShiftTol);
      if (whole) {
        fail = sf;
        if (t == 0)
          for (int i = 0; i < win; ++i) {
            wr[l + i] = wv[i] + shift;
            wi[l + i] = wv[kNsMsMinWindow + i];
          }
        nn = l - 1;
        break;
      }
      if (sf) {
        ns_ds_iteration(tm, B, l, nn, x, y, w);
        continue;
      }
      if (t == 0) ns_pair_shifts(sr, si, ns);
      tm.sync();
      ns_ms_sweep(tm, B, l, nn, sr, si, ns / 2, rt);
    }
  }
#undef HB
  tm.sync();
  return fail;
}

// norm of the upper Hessenberg band (sum of absolute entries), the scale of
// the deflation test where two diagonal entries are both zero
template <class Team, class Band>
KA_HD double ns_band_norm(Team& tm, const Band& B, int n) {
  const int t = tm.tid(), NT = tm.size();
  double anorm = 0.0;
  for (int j = t; j < n; j += NT) {
    const double* c = B.col(j);
    for (int i = 0; i <= j + 1 && i < n; ++i) anorm += fabs(c[i]);
  }
  return tm.sum(anorm);
}

// The whole eigenvalue stage by ns_ms_run on the band hb.  With fast !=
// nullptr (a band of order fast_n) and n > fast_n, the columns below fast_n
// move to fast first and the band is split there until the leading block fits
// in fast; the device does the same with LDS.
template <class Team, class SmallEig>
KA_HD int ns_qr_values_ms(Team& tm, double* hb, int n, double* wr, double* wi, double* anorm_out, double* scr,
                          const SmallEig& small_eig, double* fast, int fast_n) {
  const double anorm = ns_band_norm(tm, NsBand{hb}, n);
  if (anorm_out && tm.tid() == 0) *anorm_out = anorm;
  int nn = n - 1;
  double shift = 0.0;
  if (!fast || n <= fast_n) return ns_ms_run(tm, NsBand{hb}, nn, shift, anorm, -1, wr, wi, scr, small_eig);
  const size_t cnt = (size_t)fast_n * (fast_n + 7) / 2;          // columns 0 .. fast_n - 1 of the band
  for (size_t e = tm.tid(); e < cnt; e += tm.size()) fast[e] = hb[e];
  tm.sync();
  if (ns_ms_run(tm, NsSplitBand{fast, hb, fast_n}, nn, shift, anorm, fast_n - 1, wr, wi, scr, small_eig)) return 1;
  return ns_ms_run(tm, NsBand{fast}, nn, shift, anorm, -1, wr, wi, scr, small_eig);
}

// ---- stage 3: rank of eigenvalue c by descending real part (ties by index) ---------------
// A conjugate pair has equal real parts and consecutive indices (positive
// imaginary part first), so it keeps its order.
KA_HD inline int ns_rank(const double* wr0, int n, int c) {
  const double kc = wr0[c];
  int rank = 0;
  for (int j = 0; j < n; ++j)
    if (wr0[j] > kc || (wr0[j] == kc && j < c)) ++rank;
  return rank;
}

// largest eigenvalue modulus: the scale of the cluster gap and pivot floor
KA_HD inline double ns_scale(const double* wr, const double* wi, int n) {
  double m = 0.0;
  for (int c = 0; c < n; ++c) m = fmax(m, ns_cabs(wr[c], wi[c]));
  return m;
}

// wanted columns: nvec, plus one when column nvec - 1 is the first of a pair
KA_HD inline int ns_wanted(const double* wi_sorted, int n, int nvec) {
  return (nvec >= 1 && nvec < n && wi_sorted[nvec - 1] > 0.0) ? nvec + 1 : nvec;
}

// ---- stage 4: inverse iteration on Hh, one team per cluster ---------------------------------
// Entries are the sorted output columns c < nv with wi[c] >= 0 (a pair is one
// entry).  B = Hh - lambda I with Hh read row-wise from HT (row-major copy of
// the upper Hessenberg matrix, sub-diagonal included).  LU with row
// interchanges between neighbours only, row-oriented so that the team splits
// each row over its threads: U row j holds columns j .. n-1 at offset
// j n - j (j - 1) / 2 of the planes Ur, Ui.  ml: multipliers (re, im) and
// interchange flags, 3n.  xs: team-shared vector (re, im), 2n.
KA_HD inline size_t ns_urow(int n, int j) { return (size_t)j * n - (size_t)j * (j - 1) / 2; }
KA_HD inline size_t ns_lu_plane(int n) { return (size_t)n * (n + 1) / 2; }

KA_HD inline bool ns_is_entry(const double* wi, int c) { return c == 0 || wi[c] >= 0.0 || wi[c - 1] <= 0.0; }

// is the entry at column c the first of its cluster?  (entries in sorted order)
KA_HD inline bool ns_cluster_first(const double* wr, const double* wi, int c, double gap) {
  if (c == 0) return true;
  int p = c - 1;
  if (p > 0 && wi[p] < 0.0) --p;                    // previous entry: the pair's first column
  return ns_cabs(wr[c] - wr[p], wi[c] - wi[p]) >= gap;
}

// column of the next entry after c, or nv
KA_HD inline int ns_next_entry(const double* wi, int c, int nv) {
  const int nx = c + ((wi[c] > 0.0) ? 2 : 1);
  return nx < nv ? nx : nv;
}

// The cluster that starts at entry c_first; V: output columns, element i of
// column c at V[i * stride + c].  scale: the largest eigenvalue modulus.
template <class Team>
KA_HD void ns_invit_team(Team& tm, const double* HT, const double* hsub, int n, const double* wr, const double* wi,
                         int c_first, int nv, int stride, double scale, double* V, double* Ur, double* Ui,
                         double* ml, double* xs) {
  const int t = tm.tid(), NT = tm.size();
  const double gap = kNsClusterGap * scale;
  const double tiny = kNsEps * (scale > 0.0 ? scale : 1.0);
  const size_t S = (size_t)stride;
  double* mr = ml;
  double* mi = ml + n;
  double* fl = ml + 2 * n;
  double* xr = xs;
  double* xi = xs + n;
#define UR(j, cc) Ur[ns_urow(n, j) + (size_t)((cc) - (j))]
#define UI(j, cc) Ui[ns_urow(n, j) + (size_t)((cc) - (j))]
  for (int c = c_first; c < nv; c = ns_next_entry(wi, c, nv)) {
    if (c != c_first && ns_cluster_first(wr, wi, c, gap)) break;
    const double lr = wr[c], li = wi[c];
    const bool cplx = li > 0.0;
    // ---- LU of B = Hh - lambda I --------------------------------------------------------
    // The planes start as the upper triangle of B (row r, columns >= r), so
    // step j reads row j+1 of B from fast memory before overwriting it.
    for (int r = 0; r < n; ++r)
      for (int cc = r + t; cc < n; cc += NT) {
        UR(r, cc) = HT[(size_t)r * n + cc] - (cc == r ? lr : 0.0);
        if (cplx) UI(r, cc) = (cc == r ? -li : 0.0);
      }
    tm.sync();
    double sub_next = n > 1 ? hsub[0] : 0.0;
    for (int j = 0; j + 1 < n; ++j) {
      double ar = UR(j, j), ai = cplx ? UI(j, j) : 0.0;
      if (ns_cabs(ar, ai) < tiny) {                // keep the factorisation finite
        ar = tiny;
        ai = 0.0;
      }
      const double sub = sub_next;                  // B[j+1][j], real
      sub_next = (j + 2 < n) ? hsub[j + 1] : 0.0;   // read one step ahead
      const bool swap = fabs(sub) > ns_cabs(ar, ai);
      double l_r, l_i;
      if (swap) {
        l_r = ar / sub;
        l_i = ai / sub;
      } else {
        const double den = ar * ar + ai * ai;
        l_r = den > 0.0 ? sub * ar / den : 0.0;
        l_i = den > 0.0 ? -sub * ai / den : 0.0;
      }
      tm.sync();                                    // every thread has read the pivot
      for (int cc = j + 1 + t; cc < n; cc += NT) {
        const double br = UR(j + 1, cc), bi = cplx ? UI(j + 1, cc) : 0.0;   // row j+1 of B
        const double ur = UR(j, cc), ui = cplx ? UI(j, cc) : 0.0;
        if (swap) {
          // U row j <- B row j+1; new current row = old row - l B row j+1
          UR(j, cc) = br;
          UR(j + 1, cc) = ur - (l_r * br - l_i * bi);
          if (cplx) {
            UI(j, cc) = bi;
            UI(j + 1, cc) = ui - (l_r * bi + l_i * br);
          }
        } else {
          // new current row = B row j+1 - l U row j
          UR(j + 1, cc) = br - (l_r * ur - l_i * ui);
          if (cplx) UI(j + 1, cc) = bi - (l_r * ui + l_i * ur);
        }
      }
      if (t == 0) {
        mr[j] = l_r;
        mi[j] = l_i;
        fl[j] = swap ? 1.0 : 0.0;
        UR(j, j) = swap ? sub : ar;
        if (cplx) UI(j, j) = swap ? 0.0 : ai;
      }
      tm.sync();
    }
    if (t == 0 && ns_cabs(UR(n - 1, n - 1), cplx ? UI(n - 1, n - 1) : 0.0) < tiny) {
      UR(n - 1, n - 1) = tiny;
      if (cplx) UI(n - 1, n - 1) = 0.0;
    }
    for (int i = t; i < n; i += NT) {
      xr[i] = sym_hash_unit((uint64_t)c + 1, (uint64_t)i);
      xi[i] = cplx ? sym_hash_unit((uint64_t)c + 7919, (uint64_t)i) : 0.0;
    }
    tm.sync();
    for (int iter = 0; iter < 3; ++iter) {
      // forward: interchanges and multipliers (a short serial chain)
      if (t == 0) {
        double ar = xr[0], ai = xi[0];
        for (int j = 0; j + 1 < n; ++j) {
          double br = xr[j + 1], bi = xi[j + 1];
          if (fl[j] != 0.0) {
            const double tr = ar, ti = ai;
            ar = br;
            ai = bi;
            br = tr;
            bi = ti;
          }
          br -= mr[j] * ar - mi[j] * ai;
          bi -= mr[j] * ai + mi[j] * ar;
          xr[j] = ar;
          xi[j] = ai;
          ar = br;
          ai = bi;
        }
        xr[n - 1] = ar;
        xi[n - 1] = ai;
      }
      tm.sync();
      // back substitution by columns: x_i = x_i / U(i,i), then the rows above
      // take their share of column i (split over the team)
      for (int i = n - 1; i >= 0; --i) {
        const double sr = xr[i], si = xi[i];
        const double dr = UR(i, i), di = cplx ? UI(i, i) : 0.0;
        const double den = dr * dr + di * di;
        double qr = (sr * dr + si * di) / den, qi = (si * dr - sr * di) / den;
        tm.sync();                                  // every thread has read x_i
        if (fabs(qr) + fabs(qi) > 1e150) {          // keep the growth representable
          for (int r = t; r < n; r += NT) {
            xr[r] *= 1e-150;
            xi[r] *= 1e-150;
          }
          qr *= 1e-150;
          qi *= 1e-150;
          tm.sync();
        }
        if (t == 0) {
          xr[i] = qr;
          xi[i] = qi;
        }
        for (int r = t; r < i; r += NT) {
          const double ur = UR(r, i), ui = cplx ? UI(r, i) : 0.0;
          xr[r] -= ur * qr - ui * qi;
          xi[r] -= ur * qi + ui * qr;
        }
        tm.sync();
      }
      // orthogonalise against the cluster's earlier entries of the same kind
      for (int pass = 0; pass < 2; ++pass)
        for (int e = c_first; e < c; e = ns_next_entry(wi, e, nv)) {
          const bool ecplx = wi[e] > 0.0;
          if (ecplx != cplx) continue;
          double dr = 0.0, di = 0.0;
          for (int i = t; i < n; i += NT) {
            const double er = V[(size_t)i * S + e], ei = ecplx ? V[(size_t)i * S + e + 1] : 0.0;
            dr += er * xr[i] + ei * xi[i];
            di += er * xi[i] - ei * xr[i];
          }
          dr = tm.sum(dr);
          di = tm.sum(di);
          for (int i = t; i < n; i += NT) {
            const double er = V[(size_t)i * S + e], ei = ecplx ? V[(size_t)i * S + e + 1] : 0.0;
            xr[i] -= dr * er - di * ei;
            xi[i] -= dr * ei + di * er;
          }
          tm.sync();
        }
      double nrm = 0.0;
      for (int i = t; i < n; i += NT) nrm += xr[i] * xr[i] + xi[i] * xi[i];
      nrm = tm.sum(nrm);
      nrm = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
      for (int i = t; i < n; i += NT) {
        xr[i] *= nrm;
        xi[i] *= nrm;
      }
      tm.sync();
    }
    for (int i = t; i < n; i += NT) {
      V[(size_t)i * S + c] = xr[i];
      if (cplx) V[(size_t)i * S + c + 1] = xi[i];
    }
    tm.sync();
  }
#undef UR
#undef UI
}

}  // namespace ka
