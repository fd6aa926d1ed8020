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

KA_HD inline size_t ns_band_doubles(int n) { return (size_t)n * (n + 7) / 2 + 8; }
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

// ---- stage 1: Hessenberg reduction by a team ---------------------------------------------
// A: n x n with leading dimension ld (fast memory if available).  v, w: team
// scratch of >= n doubles each.  Team interface as in sym_core.hpp.
template <class Team>
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
      // left: A[j+1:, c] -= b v (v^T A[j+1:, c]) for c > j
      for (int c = j + 1 + t; c < n; c += NT) {
        double s0 = 0.0, s1 = 0.0;
        int i = 0;
        for (; i + 1 < m; i += 2) {
          s0 += v[i] * AH(j + 1 + i, c);
          s1 += v[i + 1] * AH(j + 2 + i, c);
        }
        if (i < m) s0 += v[i] * AH(j + 1 + i, c);
        w[c] = b * (s0 + s1);
      }
      tm.sync();
      // the rank-one updates are spread over the whole team, one element per
      // thread and pass, in memory order (each element takes the same single
      // update as in a row-by-row loop)
      const int nc = n - j - 1;
      for (int e = t; e < m * nc; e += NT) {
        const int i = e % m, c = j + 1 + e / m;
        AH(j + 1 + i, c) -= w[c] * v[i];
      }
      tm.sync();
      // right: A[r, j+1:] -= b (A[r, j+1:] v) v^T for every row
      for (int r = t; r < n; r += NT) {
        double s0 = 0.0, s1 = 0.0;
        int i = 0;
        for (; i + 1 < m; i += 2) {
          s0 += AH(r, j + 1 + i) * v[i];
          s1 += AH(r, j + 2 + i) * v[i + 1];
        }
        if (i < m) s0 += AH(r, j + 1 + i) * v[i];
        w[r] = b * (s0 + s1);
      }
      tm.sync();
      for (int e = t; e < n * m; e += NT) {
        const int r = e % n, i = e / n;
        AH(r, j + 1 + i) -= w[r] * v[i];
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

template <class Team>
KA_HD int ns_qr_values(Team& tm, double* hb, int n, double* wr, double* wi, double* anorm_out) {
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
        if (fabs(HB(l, l - 1)) <= kNsEps * s) break;
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
        tm.sync();
        for (int i = t; i <= nn; i += NT) HB(i, i) -= x;
        tm.sync();
        const double s = ns_exceptional_top(its) ? fabs(HB(l + 1, l)) + fabs(HB(l + 2, l + 1))
                                                  : fabs(HB(nn, nn - 1)) + fabs(HB(nn - 1, nn - 2));
        x = y = 0.75 * s;
        w = -0.4375 * s * s;
      }
      ++its;
      // start of the double step: two consecutive small sub-diagonal elements
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
        double xx = 0.0;
        if (k != m) {
          p = HB(k, k - 1);
          q = HB(k + 1, k - 1);
          r = notlast ? HB(k + 2, k - 1) : 0.0;
          xx = fabs(p) + fabs(q) + fabs(r);
          if (xx != 0.0) {
            const double ixx = 1.0 / xx;
            p *= ixx;
            q *= ixx;
            r *= ixx;
          }
        }
        const double s = ns_sgn(sqrt(p * p + q * q + r * r), p);
        tm.sync();
        if (s == 0.0) continue;
        if (t == 0) {
          if (k == m) {
            if (l != m) HB(k, k - 1) = -HB(k, k - 1);
          } else {
            HB(k, k - 1) = -s * xx;
          }
        }
        const double pp = p + s;
        const double is = 1.0 / s, ipp = 1.0 / pp;
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
    }
  }
  tm.sync();
#undef HB
  return fail;
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
