// Small dense symmetric eigensolve for the Rayleigh-Ritz step of the Galerkin
// method (the projected matrix of the symmetric standard form A' = L^-1 A L^-T,
// paper Sec. 3.1).  Split into stages that parallelise differently:
//   1. Householder tridiagonalisation  H = Q T Q^T  by a team of threads
//      (reflectors kept in the strictly lower part of the working copy A);
//   2. eigenvalue k of T by multisection on Sturm counts (one wave per value);
//   3. eigenvectors of T by inverse iteration with the pivoted tridiagonal
//      LU, for the wanted (largest) eigenvalues only; eigenvalues closer than
//      a gap form a cluster, handled by one thread that orthogonalises each
//      member against the ones before it after every solve, so clustered
//      vectors come out orthonormal                           (one per cluster);
//   4. back-transformation x <- Q x by the reflectors          (one per vector).
// Every function here is plain C++ usable on the host (unit tests) and on the
// device (sym.hip runs stage 1 as one workgroup, stages 2-4 as wide grids).
//
// Work layout (doubles), n = order:
//   A    n*n    column-major working copy, reflectors below the sub-diagonal
//   V    n*n    vectors interleaved: element i of vector k at V[i*n + k]
//   F    5*n*n  per-thread LU factors (when not in fast memory), interleaved
//               like V per field
//   d, e, beta, lam   4*n  (diagonal, off-diagonal, reflector coefficients,
//                           eigenvalues ascending)
//   bnd  4      Gershgorin lower / upper bound, norm estimate
//   Xw   n*n    per-thread iteration vectors when they do not fit in fast memory
#pragma once
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#ifndef KA_HD
#ifdef __HIPCC__
#define KA_HD __host__ __device__
#else
#define KA_HD
#endif
#endif
#ifndef KA_FORCEINLINE
#define KA_FORCEINLINE __attribute__((always_inline)) inline
#endif

namespace ka {

struct SymWork {
  double *A, *V, *F, *d, *e, *beta, *lam, *bnd, *Xw;
};

KA_HD inline size_t sym_tri_work_doubles(int n) { return (size_t)8 * n * n + (size_t)4 * n + 4; }

KA_HD inline SymWork sym_work_split(double* w, int n) {
  const size_t nn = (size_t)n * n;
  SymWork s;
  s.A = w;
  s.V = w + nn;
  s.F = w + 2 * nn;
  s.d = w + 7 * nn;
  s.e = s.d + n;
  s.beta = s.e + n;
  s.lam = s.beta + n;
  s.bnd = s.lam + n;
  s.Xw = s.bnd + 4;
  return s;
}

constexpr double kSymEps = 2.220446049250313e-16;
// eigenvalues closer than this (relative to the norm estimate) form a cluster
constexpr double kSymClusterGap = 1e-8;

KA_HD inline double sym_copysign(double a, double b) { return b >= 0.0 ? fabs(a) : -fabs(a); }

// ---- stage 1: tridiagonalisation by a team ---------------------------------------
// Team interface: tid(), size(), sync(), sum(x) (total over the team, returned to
// every thread).  v: team-shared scratch of >= n doubles.  A: n x n column-major
// (may live in fast memory); w: a free column of >= n doubles for the product.
// elements per thread whose loads the tridiagonalisation issues together
// (enough in flight to cover the latency of a matrix held in device memory)
constexpr int kSymBatch = 8;

template <class Team>
KA_HD void sym_tridiagonalize(Team& tm, double* A, int n, double* d, double* e, double* beta, double* v,
                              double* w) {
  const int t = tm.tid(), NT = tm.size();
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    double* col = A + (j + 1) + (size_t)j * n;      // column j below the diagonal
    double ss = 0.0;
    for (int i = t; i < m; i += NT) ss += col[i] * col[i];
    ss = tm.sum(ss);
    const double x0 = col[0];
    const double alpha = -sym_copysign(sqrt(ss), x0);
    const double v0 = x0 - alpha;
    const bool skip = !(ss > 1e-300);
    const double vtv = ss - x0 * x0 + v0 * v0;     // >= ss whenever ss > 0
    const double b = skip ? 0.0 : 2.0 / vtv;
    for (int i = t; i < m; i += NT) v[i] = (i == 0) ? v0 : col[i];
    if (t == 0) {
      d[j] = A[j + (size_t)j * n];
      e[j] = skip ? x0 : alpha;
      beta[j] = b;
    }
    tm.sync();
    if (!skip) {
      double* A22 = A + (j + 1) + (size_t)(j + 1) * n;
      // w = b A22 v: a thread per row, kSymBatch columns at a time with their
      // loads issued together (eight partial sums, added in a fixed tree)
      for (int r = t; r < m; r += NT) {
        const double* row = A22 + r;
        double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int c = 0;
        for (; c + kSymBatch - 1 < m; c += kSymBatch) {
          double a[kSymBatch];
#pragma unroll
          for (int u = 0; u < kSymBatch; ++u) a[u] = row[(size_t)(c + u) * n];
#pragma unroll
          for (int u = 0; u < kSymBatch; ++u) acc[u % 8] += a[u] * v[c + u];
        }
        for (; c < m; ++c) acc[0] += row[(size_t)c * n] * v[c];
        w[r] = b * (((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7])));
      }
      tm.sync();
      double wv = 0.0;
      for (int r = t; r < m; r += NT) wv += w[r] * v[r];
      wv = tm.sum(wv);
      const double K = 0.5 * b * wv;
      for (int r = t; r < m; r += NT) w[r] -= K * v[r];
      tm.sync();
      // A22 <- A22 - v w^T - w v^T  (= H A22 H): thread t takes row t % m in
      // the columns of its group t / m (groups of m threads; the columns of a
      // row are shared out among the groups), kSymBatch columns at a time with
      // the loads first, so that consecutive threads touch consecutive rows
      const int groups = NT >= m ? NT / m : 1;
      for (int r0 = t; r0 < groups * m; r0 += NT) {   // one pass when NT >= m, else rows r0, r0 + NT, ...
        const int r = NT >= m ? r0 % m : r0, g = NT >= m ? r0 / m : 0;
        if (r >= m) continue;
        double* row = A22 + r;
        const double vr = v[r], wr = w[r];
        int c = g;
        for (; c + (kSymBatch - 1) * groups < m; c += kSymBatch * groups) {
          double a[kSymBatch];
#pragma unroll
          for (int u = 0; u < kSymBatch; ++u) a[u] = row[(size_t)(c + u * groups) * n];
#pragma unroll
          for (int u = 0; u < kSymBatch; ++u) {
            const int cc = c + u * groups;
            row[(size_t)cc * n] = a[u] - (vr * w[cc] + wr * v[cc]);
          }
        }
        for (; c < m; c += groups) row[(size_t)c * n] -= vr * w[c] + wr * v[c];
      }
    }
    tm.sync();
    for (int i = t; i < m; i += NT) col[i] = v[i];  // reflector for the back-transformation
    tm.sync();
  }
  if (t == 0) {
    if (n >= 2) {
      d[n - 2] = A[(n - 2) + (size_t)(n - 2) * n];
      e[n - 2] = A[(n - 1) + (size_t)(n - 2) * n];
    }
    d[n - 1] = A[(n - 1) + (size_t)(n - 1) * n];
  }
  tm.sync();
}

// Blocked form of the same reduction (the split of LAPACK's latrd and syr2k):
// within a panel of nb columns the two-sided updates are deferred.  Column j
// of the panel first takes the updates of the panel's earlier columns, the
// product A22 v is corrected for them (A22 is read as stored, without them),
// and the trailing matrix takes all of the panel's updates at the panel's
// end, as one rank-2nb update.  The passes over the matrix per nb columns go
// from 3 nb to nb + 2, for a matrix held in device memory; the arithmetic is
// the same up to the order of the sums.  Team: as above, plus
// sumv(x, k, out): out[i] = sum over the team of x[i], i < k, into
// team-shared out, returned to every thread.  V, W: team-shared, nb columns of
// n doubles each (panel column s at V[s * n + r], rows r in the matrix's
// numbering, zero at and above the column's diagonal); yz: team-shared,
// >= 2 kSymNbMax doubles.
constexpr int kSymNbMax = 8;

template <class Team>
KA_HD KA_FORCEINLINE void sym_tridiagonalize_blocked(Team& tm, double* A, int n, double* d, double* e, double* beta,
                                                     double* v, double* w, double* V, double* W, double* yz, int nb) {
  const int t = tm.tid(), NT = tm.size();
  if (nb > kSymNbMax) nb = kSymNbMax;
  if (nb < 1) nb = 1;
  for (int p0 = 0; p0 + 2 < n; p0 += nb) {
    const int pend = p0 + nb < n - 2 ? p0 + nb : n - 2;   // panel columns p0 .. pend - 1
    for (int j = p0; j < pend; ++j) {
      const int sn = j - p0;                 // earlier columns of this panel
      const int m = n - j - 1;
      double* colj = A + (size_t)j * n;
      // column j, rows j .. n-1: the panel's deferred updates
      if (sn > 0) {
        for (int r = j + t; r < n; r += NT) {
          double c = colj[r];
          for (int q = 0; q < sn; ++q) c -= V[(size_t)q * n + r] * W[(size_t)q * n + j] + W[(size_t)q * n + r] * V[(size_t)q * n + j];
          colj[r] = c;
        }
        tm.sync();
      }
      double* col = colj + j + 1;             // column j below the diagonal
      double ss = 0.0;
      for (int i = t; i < m; i += NT) ss += col[i] * col[i];
      ss = tm.sum(ss);
      const double x0 = col[0];
      const double alpha = -sym_copysign(sqrt(ss), x0);
      const double v0 = x0 - alpha;
      const bool skip = !(ss > 1e-300);
      const double vtv = ss - x0 * x0 + v0 * v0;
      const double b = skip ? 0.0 : 2.0 / vtv;
      for (int i = t; i < m; i += NT) v[i] = (i == 0) ? v0 : col[i];
      if (t == 0) {
        d[j] = colj[j];
        e[j] = skip ? x0 : alpha;
        beta[j] = b;
      }
      tm.sync();
      if (!skip) {
        const double* A22 = A + (j + 1) + (size_t)(j + 1) * n;
        // p = A22 v as stored: a thread per row, kSymBatch loads in flight
        for (int r = t; r < m; r += NT) {
          const double* row = A22 + r;
          double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
          int c = 0;
          for (; c + kSymBatch - 1 < m; c += kSymBatch) {
            double a[kSymBatch];
#pragma unroll
            for (int u = 0; u < kSymBatch; ++u) a[u] = row[(size_t)(c + u) * n];
#pragma unroll
            for (int u = 0; u < kSymBatch; ++u) acc[u % 8] += a[u] * v[c + u];
          }
          for (; c < m; ++c) acc[0] += row[(size_t)c * n] * v[c];
          w[r] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        }
        // the panel's deferred part: p -= V (W^T v) + W (V^T v)
        if (sn > 0) {
          double part[2 * kSymNbMax];
#pragma unroll
          for (int q = 0; q < 2 * kSymNbMax; ++q) part[q] = 0.0;
          for (int c = t; c < m; c += NT) {
            const double vc = v[c];
            const size_t rc = (size_t)(j + 1 + c);
#pragma unroll
            for (int q = 0; q < kSymNbMax; ++q)
              if (q < sn) {
                part[q] += W[(size_t)q * n + rc] * vc;
                part[kSymNbMax + q] += V[(size_t)q * n + rc] * vc;
              }
          }
          tm.sumv(part, 2 * kSymNbMax, yz);
          for (int r = t; r < m; r += NT) {
            const size_t rr = (size_t)(j + 1 + r);
            double c = w[r];
            for (int q = 0; q < sn; ++q) c -= V[(size_t)q * n + rr] * yz[q] + W[(size_t)q * n + rr] * yz[kSymNbMax + q];
            w[r] = c;
          }
        }
        double wv = 0.0;
        for (int r = t; r < m; r += NT) {
          w[r] *= b;
          wv += w[r] * v[r];
        }
        wv = tm.sum(wv);
        const double K = 0.5 * b * wv;
        for (int r = t; r < m; r += NT) w[r] -= K * v[r];
      } else {
        for (int r = t; r < m; r += NT) w[r] = 0.0;
      }
      tm.sync();
      // panel column sn, and the reflector for the back-transformation
      for (int r = t; r < n; r += NT) {
        V[(size_t)sn * n + r] = r > j ? v[r - j - 1] : 0.0;
        W[(size_t)sn * n + r] = r > j ? w[r - j - 1] : 0.0;
      }
      for (int i = t; i < m; i += NT) col[i] = v[i];
      tm.sync();
    }
    // the trailing matrix, rows and columns pend .. n-1, takes the panel's
    // updates: A <- A - V W^T - W V^T
    const int ns = pend - p0, mt = n - pend;
#if defined(__HIP_DEVICE_COMPILE__)
    {
      // On the FP64 matrix cores: a 16 x 16 tile takes tile - L R^T with
      // L = [V W] (its rows) and R = [W V] (its columns), K = 2 kSymNbMax in
      // four v_mfma_f64_16x16x4f64 (A lane l: row l % 16, k l / 16; B lane l:
      // k l / 16, column l % 16; accumulator entry e of lane l: row
      // l / 16 + 4 e, column l % 16).  Each wave takes four tiles at a time,
      // their loads issued together; parts of tiles past the matrix are
      // neither read nor written, and panel columns past ns weigh zero.
      typedef double sym_d4 __attribute__((ext_vector_type(4)));
      constexpr int kTiles = 4;
      const int lane = t & 63, wv = t >> 6, nwv = NT >> 6;
      const int li = lane & 15, lk = lane >> 4;
      const int n16 = (mt + 15) / 16, ntl = n16 * n16;
      for (int base = wv * kTiles; base < ntl; base += nwv * kTiles) {
        sym_d4 acc[kTiles];
#pragma unroll
        for (int u = 0; u < kTiles; ++u) {
          const int tile = base + u;
          const int ti = tile % n16, tj = tile / n16;
          const int cj = tj * 16 + li;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int ri = ti * 16 + lk + 4 * e;
            acc[u][e] = (tile < ntl && ri < mt && cj < mt) ? A[(size_t)(pend + ri) + (size_t)(pend + cj) * n] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < kTiles; ++u) {
          const int tile = base + u;
          const int ti = tile % n16, tj = tile / n16;
          const int ra = ti * 16 + li, cb = tj * 16 + li;
#pragma unroll
          for (int h = 0; h < 2 * kSymNbMax / 4; ++h) {
            const int k = 4 * h + lk, q = k % kSymNbMax;
            const bool first = k < kSymNbMax;
            double av = 0.0, bv = 0.0;
            if (tile < ntl && q < ns) {
              if (ra < mt) av = -(first ? V : W)[(size_t)q * n + pend + ra];
              if (cb < mt) bv = (first ? W : V)[(size_t)q * n + pend + cb];
            }
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
          }
        }
#pragma unroll
        for (int u = 0; u < kTiles; ++u) {
          const int tile = base + u;
          const int ti = tile % n16, tj = tile / n16;
          const int cj = tj * 16 + li;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int ri = ti * 16 + lk + 4 * e;
            if (tile < ntl && ri < mt && cj < mt) A[(size_t)(pend + ri) + (size_t)(pend + cj) * n] = acc[u][e];
          }
        }
      }
    }
#else
    // thread t takes row t % mt in the columns of its group t / mt,
    // kSymBatch columns at a time
    const int groups = NT >= mt ? NT / mt : 1;
    for (int r0 = t; r0 < groups * mt; r0 += NT) {
      const int r = NT >= mt ? r0 % mt : r0, g = NT >= mt ? r0 / mt : 0;
      const size_t rr = (size_t)(pend + r);
      double vr[kSymNbMax], wr[kSymNbMax];
#pragma unroll
      for (int q = 0; q < kSymNbMax; ++q) {
        vr[q] = q < ns ? V[(size_t)q * n + rr] : 0.0;
        wr[q] = q < ns ? W[(size_t)q * n + rr] : 0.0;
      }
      double* row = A + rr + (size_t)pend * n;
      int c = g;
      for (; c + (kSymBatch - 1) * groups < mt; c += kSymBatch * groups) {
        double a[kSymBatch];
#pragma unroll
        for (int u = 0; u < kSymBatch; ++u) a[u] = row[(size_t)(c + u * groups) * n];
#pragma unroll
        for (int u = 0; u < kSymBatch; ++u) {
          const size_t cc = (size_t)(pend + c + u * groups);
          double x = a[u];
#pragma unroll
          for (int q = 0; q < kSymNbMax; ++q)
            if (q < ns) x -= vr[q] * W[(size_t)q * n + cc] + wr[q] * V[(size_t)q * n + cc];
          row[(size_t)(c + u * groups) * n] = x;
        }
      }
      for (; c < mt; c += groups) {
        const size_t cc = (size_t)(pend + c);
        double x = row[(size_t)c * n];
        for (int q = 0; q < ns; ++q) x -= vr[q] * W[(size_t)q * n + cc] + wr[q] * V[(size_t)q * n + cc];
        row[(size_t)c * n] = x;
      }
    }
#endif
    tm.sync();
  }
  if (t == 0) {
    if (n >= 2) {
      d[n - 2] = A[(n - 2) + (size_t)(n - 2) * n];
      e[n - 2] = A[(n - 1) + (size_t)(n - 2) * n];
    }
    d[n - 1] = A[(n - 1) + (size_t)(n - 1) * n];
  }
  tm.sync();
}

// Gershgorin interval and norm estimate of T (d, e)
KA_HD inline void sym_bounds(const double* d, const double* e, int n, double* bnd) {
  double lo = 1e300, hi = -1e300, tn = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    tn = fmax(tn, fabs(d[i]) + r);
  }
  if (!(tn > 0.0)) tn = 1.0;
  bnd[0] = lo - 4.0 * kSymEps * tn;
  bnd[1] = hi + 4.0 * kSymEps * tn;
  bnd[2] = tn;
  bnd[3] = 0.0;
}

// number of eigenvalues of T smaller than x (Sturm sequence of the LDL^T pivots)
KA_HD inline int sym_sturm_count(const double* d, const double* e, int n, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

// ---- stage 2: the k-th smallest eigenvalue (k = 0 .. n-1) by multisection ----------
// Each round evaluates the Sturm count at P interior points of [lo, hi] (one per
// lane on the GPU) and keeps the sub-interval where the count passes k, so the
// interval shrinks by P + 1 per round.
KA_HD inline double sym_pivmin(const double* bnd) { return 1e-280 * fmax(1.0, bnd[2] * bnd[2]); }

KA_HD inline bool sym_section_done(double lo, double hi, const double* bnd) {
  return hi - lo <= 2.0 * kSymEps * fmax(fabs(lo), fabs(hi)) + 1e-3 * kSymEps * bnd[2];
}

KA_HD inline double sym_section_point(double lo, double hi, int t, int P) {
  return lo + (hi - lo) * ((double)(t + 1) / (double)(P + 1));
}

// mask bit t set when count(point t) > k
KA_HD inline void sym_section_narrow(double& lo, double& hi, uint64_t mask, int P) {
  const double lo0 = lo, hi0 = hi;
  if (mask == 0) {
    lo = sym_section_point(lo0, hi0, P - 1, P);
  } else {
    const int f = __builtin_ctzll(mask);
    hi = sym_section_point(lo0, hi0, f, P);
    if (f > 0) lo = sym_section_point(lo0, hi0, f - 1, P);
  }
}

constexpr int kSymSectionRounds = 32;

KA_HD inline double sym_hash_unit(uint64_t a, uint64_t b) {
  uint64_t z = a * 0x9E3779B97F4A7C15ull + b + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0) - 0.5;
}

// Only the leading nvec eigenvectors (the largest eigenvalues, indices
// n - nvec .. n - 1 of the ascending order) are computed.  A cluster is
// walked from its largest member down, so it can stop at the first index that
// is not wanted.

// is eigenvalue k the largest of its cluster?  (lam ascending)
KA_HD inline bool sym_cluster_top(const double* lam, int n, int k, const double* bnd) {
  return k == n - 1 || lam[k + 1] - lam[k] >= kSymClusterGap * bnd[2];
}

// ---- stage 3: inverse iteration, cluster with largest member ktop, down to kstop ----
// Working storage of the calling thread: the iterated vector at xw[i * xs],
// the five LU fields at fw[f * fs + i * is] (fast memory on the GPU when they
// fit); finished vectors are stored in V.
KA_HD inline void sym_inverse_iteration(const double* d, const double* e, int n, const double* lam, int ktop,
                                        int kstop, const double* bnd, double* V, double* fw, size_t fs, int is,
                                        double* xw, int xs) {
  const double tn = bnd[2];
  const double gap = kSymClusterGap * tn;
  const double tiny = kSymEps * tn;
  int c0 = ktop;
  while (c0 > kstop && lam[c0] - lam[c0 - 1] < gap) --c0;
  double sig_prev = 1e300;
  for (int k = ktop; k >= c0; --k) {
#define XK(i) xw[(size_t)(i) * xs]
#define FK(f, i) fw[(f) * fs + (size_t)(i) * is]
    // distinct shifts inside a cluster
    double sig = lam[k];
    if (k < ktop && sig > sig_prev - 10.0 * tiny) sig = sig_prev - 10.0 * tiny;
    sig_prev = sig;
    // LU of T - sig I with partial pivoting; fields: 0 U diagonal, 1 and 2 the
    // two super-diagonals of U, 3 multiplier, 4 row interchange flag
    double a = d[0] - sig, bs = n > 1 ? e[0] : 0.0, cs = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
      const double sub = e[i], dn = d[i + 1] - sig, en = (i + 2 < n) ? e[i + 1] : 0.0;
      if (fabs(a) >= fabs(sub)) {
        const double l = (a != 0.0) ? sub / a : 0.0;
        FK(0, i) = a;
        FK(1, i) = bs;
        FK(2, i) = cs;
        FK(3, i) = l;
        FK(4, i) = 0.0;
        a = dn - l * bs;
        bs = en - l * cs;
      } else {
        const double l = a / sub;
        FK(0, i) = sub;
        FK(1, i) = dn;
        FK(2, i) = en;
        FK(3, i) = l;
        FK(4, i) = 1.0;
        a = bs - l * dn;
        bs = cs - l * en;
      }
      cs = 0.0;
    }
    FK(0, n - 1) = a;
    FK(1, n - 1) = 0.0;
    FK(2, n - 1) = 0.0;
    // store reciprocal pivots (tiny ones raised to the floor)
    for (int i = 0; i < n; ++i) {
      double u = FK(0, i);
      if (fabs(u) < tiny) u = sym_copysign(tiny, u);
      FK(0, i) = 1.0 / u;
    }
    for (int i = 0; i < n; ++i) XK(i) = sym_hash_unit((uint64_t)k + 1, (uint64_t)i);
    for (int iter = 0; iter < 3; ++iter) {
      // forward: row interchanges and multipliers (running value in a register)
      double xi = XK(0);
      for (int i = 0; i + 1 < n; ++i) {
        double xn = XK(i + 1);
        if (FK(4, i) != 0.0) {
          const double tmp = xi;
          xi = xn;
          xn = tmp;
        }
        xn -= FK(3, i) * xi;
        XK(i) = xi;
        xi = xn;
      }
      XK(n - 1) = xi;
      // back substitution with the three bands of U
      double x1 = 0.0, x2 = 0.0;   // x[i+1], x[i+2]
      for (int i = n - 1; i >= 0; --i) {
        double s = (XK(i) - FK(1, i) * x1 - FK(2, i) * x2) * FK(0, i);
        if (fabs(s) > 1e150) {                      // keep the growth representable
          for (int r = i + 1; r < n; ++r) XK(r) *= 1e-150;
          for (int r = 0; r < i; ++r) XK(r) *= 1e-150;
          s *= 1e-150;
          x1 *= 1e-150;
          x2 *= 1e-150;
        }
        XK(i) = s;
        x2 = x1;
        x1 = s;
      }
      // orthogonalise against the cluster's members computed before (two
      // passes).  Elements of a stored vector are n apart, so every one is
      // its own cache line: they are loaded 16 at a time, all in flight
      // together, before any is used (four partial sums over i mod 4).
      for (int pass = 0; pass < (k < ktop ? 2 : 0); ++pass)
        for (int j = k + 1; j <= ktop; ++j) {
          const double* vj = V + j;
          double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
          int i = 0;
          for (; i + 15 < n; i += 16) {
            double v[16];
            for (int u = 0; u < 16; ++u) v[u] = vj[(size_t)(i + u) * n];
            for (int u = 0; u < 16; u += 4) {
              d0 += XK(i + u) * v[u];
              d1 += XK(i + u + 1) * v[u + 1];
              d2 += XK(i + u + 2) * v[u + 2];
              d3 += XK(i + u + 3) * v[u + 3];
            }
          }
          for (; i + 3 < n; i += 4) {
            d0 += XK(i) * vj[(size_t)i * n];
            d1 += XK(i + 1) * vj[(size_t)(i + 1) * n];
            d2 += XK(i + 2) * vj[(size_t)(i + 2) * n];
            d3 += XK(i + 3) * vj[(size_t)(i + 3) * n];
          }
          for (; i < n; ++i) d0 += XK(i) * vj[(size_t)i * n];
          const double dot = (d0 + d1) + (d2 + d3);
          for (i = 0; i + 15 < n; i += 16) {
            double v[16];
            for (int u = 0; u < 16; ++u) v[u] = vj[(size_t)(i + u) * n];
            for (int u = 0; u < 16; ++u) XK(i + u) -= dot * v[u];
          }
          for (; i < n; ++i) XK(i) -= dot * vj[(size_t)i * n];
        }
      double nr = 0.0;
      for (int i = 0; i < n; ++i) nr += XK(i) * XK(i);
      nr = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
      for (int i = 0; i < n; ++i) XK(i) *= nr;
    }
    for (int i = 0; i < n; ++i) V[(size_t)i * n + k] = XK(i);
#undef XK
#undef FK
  }
}

// ---- stage 4: x <- Q x = H_0 H_1 ... H_{n-3} x, element i of x at x[i * stride] ----
// one reflector: y <- (I - b v v^T) y, y and v of length m
KA_HD inline void sym_reflect(const double* v, int m, double b, double* y, int stride) {
  double s0 = 0.0, s1 = 0.0;
  int i = 0;
  for (; i + 1 < m; i += 2) {
    s0 += v[i] * y[(size_t)i * stride];
    s1 += v[i + 1] * y[(size_t)(i + 1) * stride];
  }
  if (i < m) s0 += v[i] * y[(size_t)i * stride];
  const double s = b * (s0 + s1);
  for (i = 0; i < m; ++i) y[(size_t)i * stride] -= s * v[i];
}

KA_HD inline void sym_back_transform(const double* A, const double* beta, int n, double* x, int stride) {
  for (int j = n - 3; j >= 0; --j)
    if (beta[j] != 0.0) sym_reflect(A + (j + 1) + (size_t)j * n, n - j - 1, beta[j], x + (size_t)(j + 1) * stride, stride);
}

}  // namespace ka
