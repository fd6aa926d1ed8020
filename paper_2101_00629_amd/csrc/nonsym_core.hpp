// Small dense non-symmetric eigensolve (real Schur form and eigenvectors),
// written once for a "team" of cooperating lanes so that the same code runs
// as one GPU wave (nonsym.hip) and as a single host thread (unit tests).
//
//   1. Householder reduction of H to upper Hessenberg form, H = Q0 Hh Q0^T.
//   2. Francis double-shift QR iteration on Hh (Golub & Van Loan, Sec. 7.5),
//      accumulating the orthogonal transformations: Hh = Q1 T Q1^T with T
//      quasi upper triangular (real Schur form).
//   3. Eigenvectors of T by back substitution, one eigenvalue per lane,
//      complex pairs in real arithmetic; then V = Q0 Q1 Y.
//   4. Sort by descending real part; normalise (unit 2-norm per real vector,
//      |re|^2 + |im|^2 = 1 per complex pair; re and im in consecutive columns).
// status: 0 ok, 1 the QR iteration did not converge.
//
// Team interface: tid(), size(), sync(), sum(x) (over all lanes), scratch
// (>= 6n doubles shared by the team).  work: nonsym_work_doubles(n) doubles;
// Abuf: optional n x n buffer in faster memory for the working matrix.
#pragma once
#include <math.h>
#include <stdint.h>

#ifndef KA_HD
#ifdef __HIPCC__
#define KA_HD __host__ __device__
#else
#define KA_HD
#endif
#endif

namespace ka {

KA_HD inline size_t nonsym_work_doubles(int n) { return (size_t)4 * n * n + 8 * (size_t)n; }

KA_HD inline double ns_sgn(double a, double b) { return b >= 0.0 ? fabs(a) : -fabs(a); }

#define AT(M, i, j) M[(i) + (int64_t)(j) * n]

template <class Team>
KA_HD void nonsym_core(Team& tm, const double* H, int n, int ldh, double* wr_out, double* wi_out, double* S,
                       int lds, double* work, int* status, double* Abuf = nullptr) {
  double* A = Abuf ? Abuf : work;            // n x n: Hessenberg, then Schur form T (fast memory if given)
  double* Zm = work + (size_t)n * n;         // accumulated orthogonal transformations
  double* Yv = work + (size_t)2 * n * n;     // eigenvectors of T (columns)
  double* Vv = work + (size_t)3 * n * n;     // Zm * Yv
  double* wr = work + (size_t)4 * n * n;
  double* wi = wr + n;
  double* nrm = wi + n;
  double* key = nrm + n;
  double* v = tm.scratch;
  const int t = tm.tid();
  const int NT = tm.size();
  const double eps = 2.220446049250313e-16;

  for (int64_t e = t; e < (int64_t)n * n; e += NT) {
    const int i = (int)(e % n), j = (int)(e / n);
    A[e] = H[i + (int64_t)j * ldh];
    Zm[e] = (i == j) ? 1.0 : 0.0;
  }
  tm.sync();

  // ---- 1. Hessenberg reduction ------------------------------------------
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;                 // length of x = A[j+1:n, j]
    double ss = 0.0;
    for (int i = t; i < m; i += NT) ss += AT(A, j + 1 + i, j) * AT(A, j + 1 + i, j);
    ss = tm.sum(ss);
    const double x0 = AT(A, j + 1, j);
    const double alpha = -ns_sgn(sqrt(ss), x0);
    const double vtv = ss - x0 * x0 + (x0 - alpha) * (x0 - alpha);
    if (ss == 0.0 || vtv <= 1e-300) continue;
    for (int i = t; i < m; i += NT) v[i] = (i == 0) ? x0 - alpha : AT(A, j + 1 + i, j);
    tm.sync();
    const double beta = 2.0 / vtv;
    // left: A[j+1:, c] -= beta v (v^T A[j+1:, c]) for c >= j
    for (int c = j + t; c < n; c += NT) {
      double w = 0.0;
      for (int i = 0; i < m; ++i) w += v[i] * AT(A, j + 1 + i, c);
      w *= beta;
      for (int i = 0; i < m; ++i) AT(A, j + 1 + i, c) -= w * v[i];
    }
    tm.sync();
    // right: A[r, j+1:] -= beta (A[r, j+1:] v) v^T for all rows; same for Zm
    for (int r = t; r < n; r += NT) {
      double w = 0.0, wz = 0.0;
      for (int i = 0; i < m; ++i) {
        w += AT(A, r, j + 1 + i) * v[i];
        wz += AT(Zm, r, j + 1 + i) * v[i];
      }
      w *= beta;
      wz *= beta;
      for (int i = 0; i < m; ++i) {
        AT(A, r, j + 1 + i) -= w * v[i];
        AT(Zm, r, j + 1 + i) -= wz * v[i];
      }
    }
    tm.sync();
    for (int i = t; i < m; i += NT)
      if (i > 0) AT(A, j + 1 + i, j) = 0.0;
    tm.sync();
  }

  // norm of the Hessenberg matrix (for tolerances)
  double anorm = 0.0;
  for (int64_t e = t; e < (int64_t)n * n; e += NT) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i <= j + 1) anorm += fabs(A[e]);
  }
  anorm = tm.sum(anorm);

  // ---- 2. Francis double-shift QR ------------------------------------------
  // Scalar control flow is identical in every lane (all lanes read the same
  // global values after a barrier); row / column updates are split over lanes.
  int nn = n - 1;
  double shift = 0.0;
  int fail = 0;
  while (nn >= 0 && !fail) {
    int its = 0;
    while (true) {
      tm.sync();
      int l;
      for (l = nn; l >= 1; --l) {
        double s = fabs(AT(A, l - 1, l - 1)) + fabs(AT(A, l, l));
        if (s == 0.0) s = anorm;
        if (fabs(AT(A, l, l - 1)) <= eps * s) break;
      }
      if (l >= 1) {
        tm.sync();
        if (t == 0) AT(A, l, l - 1) = 0.0;
        tm.sync();
      }
      double x = AT(A, nn, nn);
      if (l == nn) {                               // one real root
        tm.sync();
        if (t == 0) {
          AT(A, nn, nn) = x + shift;
          wr[nn] = x + shift;
          wi[nn] = 0.0;
        }
        --nn;
        break;
      }
      double y = AT(A, nn - 1, nn - 1);
      double w = AT(A, nn, nn - 1) * AT(A, nn - 1, nn);
      if (l == nn - 1) {                           // a 2 x 2 block
        const double p = 0.5 * (y - x);
        const double q = p * p + w;
        double z = sqrt(fabs(q));
        x += shift;
        tm.sync();
        if (t == 0) {
          AT(A, nn, nn) = x;
          AT(A, nn - 1, nn - 1) = y + shift;
        }
        tm.sync();
        if (q >= 0.0) {                            // real pair: rotate to triangular
          z = p + ns_sgn(z, p);
          const double r1 = x + z;
          const double r2 = (z != 0.0) ? x - w / z : x + z;
          const double xs = AT(A, nn, nn - 1);
          const double s = fabs(xs) + fabs(z);
          double pp = xs / s, qq = z / s;
          const double r = sqrt(pp * pp + qq * qq);
          pp /= r;
          qq /= r;
          tm.sync();
          for (int j = nn - 1 + t; j < n; j += NT) {
            const double zz = AT(A, nn - 1, j);
            AT(A, nn - 1, j) = qq * zz + pp * AT(A, nn, j);
            AT(A, nn, j) = qq * AT(A, nn, j) - pp * zz;
          }
          tm.sync();
          for (int i = t; i <= nn; i += NT) {
            const double zz = AT(A, i, nn - 1);
            AT(A, i, nn - 1) = qq * zz + pp * AT(A, i, nn);
            AT(A, i, nn) = qq * AT(A, i, nn) - pp * zz;
          }
          for (int i = t; i < n; i += NT) {
            const double zz = AT(Zm, i, nn - 1);
            AT(Zm, i, nn - 1) = qq * zz + pp * AT(Zm, i, nn);
            AT(Zm, i, nn) = qq * AT(Zm, i, nn) - pp * zz;
          }
          tm.sync();
          if (t == 0) {
            AT(A, nn, nn - 1) = 0.0;
            // eigenvalues are the diagonal of the now triangular block
            wr[nn - 1] = AT(A, nn - 1, nn - 1);
            wr[nn] = AT(A, nn, nn);
            wi[nn - 1] = wi[nn] = 0.0;
            (void)r1;
            (void)r2;
          }
        } else {                                   // complex pair
          if (t == 0) {
            wr[nn - 1] = wr[nn] = x + p;
            wi[nn - 1] = z;
            wi[nn] = -z;
          }
        }
        nn -= 2;
        break;
      }
      if (its >= 60) {
        fail = 1;
        break;
      }
      if (its == 10 || its == 20 || its == 40) {   // exceptional shift
        shift += x;
        tm.sync();
        for (int i = t; i <= nn; i += NT) AT(A, i, i) -= x;
        tm.sync();
        const double s = fabs(AT(A, nn, nn - 1)) + fabs(AT(A, nn - 1, nn - 2));
        x = y = 0.75 * s;
        w = -0.4375 * s * s;
      }
      ++its;
      // two consecutive small sub-diagonal elements
      int m;
      double p = 0.0, q = 0.0, r = 0.0, z = 0.0;
      for (m = nn - 2; m >= l; --m) {
        z = AT(A, m, m);
        r = x - z;
        const double s0 = y - z;
        p = (r * s0 - w) / AT(A, m + 1, m) + AT(A, m, m + 1);
        q = AT(A, m + 1, m + 1) - z - r - s0;
        r = AT(A, m + 2, m + 1);
        const double s = fabs(p) + fabs(q) + fabs(r);
        p /= s;
        q /= s;
        r /= s;
        if (m == l) break;
        const double u = fabs(AT(A, m, m - 1)) * (fabs(q) + fabs(r));
        const double vv = fabs(p) * (fabs(AT(A, m - 1, m - 1)) + fabs(z) + fabs(AT(A, m + 1, m + 1)));
        if (u <= eps * vv) break;
      }
      tm.sync();
      for (int i = m + 2 + t; i <= nn; i += NT) {
        AT(A, i, i - 2) = 0.0;
        if (i != m + 2) AT(A, i, i - 3) = 0.0;
      }
      tm.sync();
      // double QR step.  The transformations of the accumulated Schur vectors
      // Zm are logged per bulge position and applied after the sweep, one
      // row per lane with a sliding window of three columns, so the sweep
      // does not wait on a memory round trip of Zm per position.
      double* zlog = v;   // 6 doubles per position: x1, y1, z1, q1, r1, flag
      for (int k = m; k <= nn - 1; ++k) {
        const bool notlast = (k != nn - 1);
        double xx = 0.0;
        if (k != m) {
          p = AT(A, k, k - 1);
          q = AT(A, k + 1, k - 1);
          r = notlast ? AT(A, k + 2, k - 1) : 0.0;
          xx = fabs(p) + fabs(q) + fabs(r);
          if (xx != 0.0) {
            p /= xx;
            q /= xx;
            r /= xx;
          }
        }
        const double s = ns_sgn(sqrt(p * p + q * q + r * r), p);
        double* e = zlog + 6 * (k - m);
        if (s == 0.0) {
          tm.sync();
          if (t == 0) e[5] = 0.0;   // no transformation at this position
          continue;
        }
        tm.sync();
        const double pp = p + s;
        const double x1 = pp / s, y1 = q / s, z1 = r / s;
        const double q1 = q / pp, r1 = r / pp;
        if (t == 0) {
          if (k == m) {
            if (l != m) AT(A, k, k - 1) = -AT(A, k, k - 1);
          } else {
            AT(A, k, k - 1) = -s * xx;
          }
          e[0] = x1;
          e[1] = y1;
          e[2] = z1;
          e[3] = q1;
          e[4] = r1;
          e[5] = 1.0;
        }
        tm.sync();
        // rows k, k+1, (k+2) over columns k..n-1
        for (int j = k + t; j < n; j += NT) {
          double pv = AT(A, k, j) + q1 * AT(A, k + 1, j);
          if (notlast) {
            pv += r1 * AT(A, k + 2, j);
            AT(A, k + 2, j) -= pv * z1;
          }
          AT(A, k + 1, j) -= pv * y1;
          AT(A, k, j) -= pv * x1;
        }
        tm.sync();
        const int imax = (nn < k + 3) ? nn : k + 3;
        for (int i = t; i <= imax; i += NT) {
          double pv = x1 * AT(A, i, k) + y1 * AT(A, i, k + 1);
          if (notlast) {
            pv += z1 * AT(A, i, k + 2);
            AT(A, i, k + 2) -= pv * r1;
          }
          AT(A, i, k + 1) -= pv * q1;
          AT(A, i, k) -= pv;
        }
        tm.sync();
      }
      // apply the sweep's logged transformations to the rows of Zm
      tm.sync();
      for (int i = t; i < n; i += NT) {
        double c0 = AT(Zm, i, m), c1 = AT(Zm, i, m + 1), c2 = AT(Zm, i, m + 2);
        for (int k = m; k <= nn - 1; ++k) {
          const double* e = zlog + 6 * (k - m);
          if (e[5] != 0.0) {
            double pv = e[0] * c0 + e[1] * c1;
            if (k != nn - 1) {
              pv += e[2] * c2;
              c2 -= pv * e[4];
            }
            c1 -= pv * e[3];
            c0 -= pv;
          }
          AT(Zm, i, k) = c0;
          c0 = c1;
          c1 = c2;
          c2 = (k + 3 <= nn) ? AT(Zm, i, k + 3) : 0.0;
        }
        AT(Zm, i, nn) = c0;
      }
      tm.sync();
    }
  }
  tm.sync();
  if (fail) {
    if (t == 0) *status = 1;
    return;
  }

  // ---- 3. eigenvectors of T by back substitution (one eigenvalue per lane) --
  double tnorm = 0.0;
  for (int64_t e = t; e < (int64_t)n * n; e += NT) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i <= j + 1) tnorm += fabs(A[e]);
    Yv[e] = 0.0;
  }
  tnorm = tm.sum(tnorm);
  tm.sync();
  const double small = eps * (tnorm > 0.0 ? tnorm : 1.0);
  for (int c = t; c < n; c += NT) {
    const double p = wr[c], q = wi[c];
    if (q == 0.0) {
      // real eigenvalue p: solve (T - p I) y = 0 with y[c] = 1, y[i > c] = 0
      AT(Yv, c, c) = 1.0;
      for (int i = c - 1; i >= 0; --i) {
        const bool second_of_pair = (i > 0) && (wi[i] < 0.0);
        if (second_of_pair) {
          // 2x2 diagonal block (i-1, i): solve the coupled pair
          const int i0 = i - 1;
          double r0 = 0.0, r1 = 0.0;
          for (int j = i + 1; j <= c; ++j) {
            r0 += AT(A, i0, j) * AT(Yv, j, c);
            r1 += AT(A, i, j) * AT(Yv, j, c);
          }
          const double a = AT(A, i0, i0) - p, b = AT(A, i0, i), cc = AT(A, i, i0), d = AT(A, i, i) - p;
          double det = a * d - b * cc;
          if (det == 0.0) det = small;
          AT(Yv, i0, c) = (-r0 * d + r1 * b) / det;
          AT(Yv, i, c) = (-r1 * a + r0 * cc) / det;
          --i;
        } else {
          double r = 0.0;
          for (int j = i + 1; j <= c; ++j) r += AT(A, i, j) * AT(Yv, j, c);
          double den = AT(A, i, i) - p;
          if (den == 0.0) den = small;
          AT(Yv, i, c) = -r / den;
        }
      }
    } else if (q < 0.0) {
      // complex pair (c-1, c): eigenvalue lambda = p + i|q| belongs to the
      // 2x2 block; eigenvector u + i v with components for indices <= c.
      const int c0 = c - 1;
      const double lr = p, li = -q;   // li > 0
      // choose the block component: solve (B - lambda I) [a; b] = 0 with b = 1
      const double b00 = AT(A, c0, c0), b01 = AT(A, c0, c), b10 = AT(A, c, c0);
      (void)b10;
      // row 0: (b00 - lambda) a + b01 * 1 = 0  ->  a = -b01 / (b00 - lambda)
      const double dr = b00 - lr, di = -li;
      const double den = dr * dr + di * di;
      double ar = -b01 * dr / (den > 0 ? den : small), ai = b01 * di / (den > 0 ? den : small);
      AT(Yv, c0, c0) = ar;
      AT(Yv, c0, c) = ai;
      AT(Yv, c, c0) = 1.0;
      AT(Yv, c, c) = 0.0;
      for (int i = c0 - 1; i >= 0; --i) {
        const bool second_of_pair = (i > 0) && (wi[i] < 0.0);
        if (second_of_pair) {
          const int i0 = i - 1;
          double r0r = 0.0, r0i = 0.0, r1r = 0.0, r1i = 0.0;
          for (int j = i + 1; j <= c; ++j) {
            r0r += AT(A, i0, j) * AT(Yv, j, c0);
            r0i += AT(A, i0, j) * AT(Yv, j, c);
            r1r += AT(A, i, j) * AT(Yv, j, c0);
            r1i += AT(A, i, j) * AT(Yv, j, c);
          }
          // [a - lam, b; cc, d - lam] [y0; y1] = -[r0; r1]  (complex)
          const double ar_ = AT(A, i0, i0) - lr, ai_ = -li, b = AT(A, i0, i), cc = AT(A, i, i0);
          const double dr_ = AT(A, i, i) - lr, di_ = -li;
          // det = (a-lam)(d-lam) - b cc
          double detr = ar_ * dr_ - ai_ * di_ - b * cc, deti = ar_ * di_ + ai_ * dr_;
          double dd = detr * detr + deti * deti;
          if (dd == 0.0) {
            detr = small;
            dd = small * small;
          }
          // y0 = (-r0 (d-lam) + b r1) / det ; y1 = (-r1 (a-lam) + cc r0) / det
          const double n0r = -(r0r * dr_ - r0i * di_) + b * r1r, n0i = -(r0r * di_ + r0i * dr_) + b * r1i;
          const double n1r = -(r1r * ar_ - r1i * ai_) + cc * r0r, n1i = -(r1r * ai_ + r1i * ar_) + cc * r0i;
          AT(Yv, i0, c0) = (n0r * detr + n0i * deti) / dd;
          AT(Yv, i0, c) = (n0i * detr - n0r * deti) / dd;
          AT(Yv, i, c0) = (n1r * detr + n1i * deti) / dd;
          AT(Yv, i, c) = (n1i * detr - n1r * deti) / dd;
          --i;
        } else {
          double rr = 0.0, ri = 0.0;
          for (int j = i + 1; j <= c; ++j) {
            rr += AT(A, i, j) * AT(Yv, j, c0);
            ri += AT(A, i, j) * AT(Yv, j, c);
          }
          // (T_ii - lambda) y = -r
          const double er = AT(A, i, i) - lr, ei = -li;
          double dd = er * er + ei * ei;
          if (dd == 0.0) dd = small * small;
          AT(Yv, i, c0) = (-rr * er - ri * ei) / dd;
          AT(Yv, i, c) = (-ri * er + rr * ei) / dd;
        }
      }
    }
  }
  tm.sync();
  // V = Zm * Yv
  for (int64_t e = t; e < (int64_t)n * n; e += NT) {
    const int i = (int)(e % n), j = (int)(e / n);
    double s = 0.0;
    for (int k2 = 0; k2 < n; ++k2) s += AT(Zm, i, k2) * AT(Yv, k2, j);
    Vv[e] = s;
  }
  tm.sync();
  // norms: real vectors individually, complex pairs jointly
  for (int c = t; c < n; c += NT) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += AT(Vv, i, c) * AT(Vv, i, c);
    nrm[c] = s;
  }
  tm.sync();
  for (int c = t; c < n; c += NT) {
    if (wi[c] > 0.0 && c + 1 < n) nrm[c] = nrm[c + 1] = nrm[c] + nrm[c + 1];
  }
  tm.sync();
  // sort by descending real part; a complex pair stays together (re first)
  for (int c = t; c < n; c += NT) key[c] = wr[c];
  tm.sync();
  for (int c = t; c < n; c += NT) {
    const double kc = key[c];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double kj = key[j];
      if (kj > kc || (kj == kc && j < c)) ++rank;
    }
    wr_out[rank] = wr[c];
    wi_out[rank] = wi[c];
    const double sc = nrm[c] > 0.0 ? 1.0 / sqrt(nrm[c]) : 0.0;
    for (int i = 0; i < n; ++i) S[i + (int64_t)rank * lds] = AT(Vv, i, c) * sc;
  }
  if (t == 0) *status = 0;
}

#undef AT

}  // namespace ka
