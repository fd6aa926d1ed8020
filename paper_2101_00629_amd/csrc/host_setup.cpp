// Host-side FP64 set-up (see host_setup.hpp).
#include "host_setup.hpp"

#include <algorithm>
#include <utility>
#include <cmath>
#include <stdexcept>

namespace ka {

Vec open_knots(int p, int nel, int mult) {
  Vec t;
  for (int i = 0; i <= p; ++i) t.push_back(0.0);
  for (int e = 1; e < nel; ++e)
    for (int m = 0; m < mult; ++m) t.push_back((double)e / nel);
  for (int i = 0; i <= p; ++i) t.push_back(1.0);
  return t;
}

Vec analysis_knots(int p, int nel, int mult, const Vec& lines, int line_mult) {
  std::vector<std::pair<double, int>> inner;
  for (int e = 1; e < nel; ++e) inner.push_back({(double)e / nel, mult});
  for (double c : lines) {
    bool merged = false;
    for (auto& b : inner)
      if (std::fabs(b.first - c) <= 1e-12) {
        b = {c, line_mult};
        merged = true;
      }
    if (!merged) inner.push_back({c, line_mult});
  }
  std::sort(inner.begin(), inner.end());
  Vec t(p + 1, 0.0);
  for (const auto& b : inner)
    for (int m = 0; m < b.second; ++m) t.push_back(b.first);
  for (int i = 0; i <= p; ++i) t.push_back(1.0);
  return t;
}

int num_basis(const Vec& t, int p) { return (int)t.size() - p - 1; }

// Knot span s with t[s] <= x < t[s+1] (left: t[s] < x <= t[s+1], the limit
// from the left); the right end belongs to the last span, the left end to
// the first.
static int find_span(const Vec& t, int p, double x, bool left = false) {
  const int n = num_basis(t, p);
  if (x >= t[n]) return n - 1;
  if (x <= t[p]) return p;
  int lo = p, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (left ? x <= t[mid] : x < t[mid]) hi = mid; else lo = mid;
  }
  return lo;
}

// The p+1 non-zero B-splines B_{s-p..s}(x) by the triangular recurrence.
static void nonzero_basis(const Vec& t, int p, int s, double x, double* N) {
  double left[32], right[32];
  N[0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    left[j] = x - t[s + 1 - j];
    right[j] = t[s + j] - x;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      const double tmp = N[r] / (right[r + 1] + left[j - r]);
      N[r] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    N[j] = saved;
  }
}

void bspline_row(const Vec& t, int p, double x, double* row, bool left) {
  const int n = num_basis(t, p);
  std::fill(row, row + n, 0.0);
  double N[32];
  const int s = find_span(t, p, x, left);
  nonzero_basis(t, p, s, x, N);
  for (int r = 0; r <= p; ++r) row[s - p + r] = N[r];
}

Mat bspline_matrix(const Vec& t, int p, const Vec& x, const std::vector<char>* left) {
  Mat B((int)x.size(), num_basis(t, p));
  for (size_t a = 0; a < x.size(); ++a) bspline_row(t, p, x[a], &B.a[a * B.cols], left && (*left)[a]);
  return B;
}

Vec greville(const Vec& t, int p) {
  const int n = num_basis(t, p);
  Vec g(n);
  for (int i = 0; i < n; ++i) {
    double s = 0;
    for (int k = 1; k <= p; ++k) s += t[i + k];
    // p equal knots: the abscissa is that knot exactly (the rounded mean may
    // miss it, and a C^-1 abscissa must sit on its knot)
    g[i] = t[i + 1] == t[i + p] ? t[i + 1] : s / p;
  }
  return g;
}

std::vector<char> greville_left(const Vec& t, int p) {
  const Vec g = greville(t, p);
  std::vector<char> left(g.size(), 0);
  for (size_t i = 0; i < g.size(); ++i) left[i] = g[i] == t[i + p + 1] && t[i + p + 1] < t.back();
  return left;
}

void gauss_legendre(int q, double a, double b, Vec& x, Vec& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;            // Legendre recurrence
      for (int k = 2; k <= q; ++k) {
        const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = z; p0 = 1.0; }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged root
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= q; ++k) {
      const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (q == 1) { p1 = z; p0 = 1.0; }
    dp = q * (z * p1 - p0) / (z * z - 1.0);
    // ascending order on [a,b]
    x[q - 1 - i] = a + (b - a) * (z + 1.0) / 2.0;
    w[q - 1 - i] = (b - a) / ((1.0 - z * z) * dp * dp);
  }
}

void element_gauss(const Vec& t, int q, Vec& x, Vec& w) {
  x.clear();
  w.clear();
  Vec xe, we;
  for (size_t k = 0; k + 1 < t.size(); ++k) {
    if (t[k + 1] > t[k]) {
      gauss_legendre(q, t[k], t[k + 1], xe, we);
      x.insert(x.end(), xe.begin(), xe.end());
      w.insert(w.end(), we.begin(), we.end());
    }
  }
}

Mat mass_matrix(const Vec& ta, int pa, const Vec& tb, int pb) {
  Vec x, w;
  element_gauss(ta, (pa + pb) / 2 + 1, x, w);
  Mat Ba = bspline_matrix(ta, pa, x), Bb = bspline_matrix(tb, pb, x);
  Mat Z(Ba.cols, Bb.cols);
  for (size_t g = 0; g < x.size(); ++g)
    for (int i = 0; i < Ba.cols; ++i) {
      const double bi = Ba(g, i) * w[g];
      if (bi == 0.0) continue;
      for (int j = 0; j < Bb.cols; ++j) Z(i, j) += bi * Bb(g, j);
    }
  return Z;
}

bool cholesky_lower(const Mat& A, Mat& L) {
  const int n = A.rows;
  L = Mat(n, n);
  for (int j = 0; j < n; ++j) {
    double d = A(j, j);
    for (int k = 0; k < j; ++k) d -= L(j, k) * L(j, k);
    if (!(d > 0)) return false;
    L(j, j) = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double s = A(i, j);
      for (int k = 0; k < j; ++k) s -= L(i, k) * L(j, k);
      L(i, j) = s / L(j, j);
    }
  }
  return true;
}

Mat lower_inverse(const Mat& L) {
  const int n = L.rows;
  Mat X(n, n);
  for (int c = 0; c < n; ++c) {          // solve L x = e_c
    for (int i = c; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= L(i, k) * X(k, c);
      X(i, c) = s / L(i, i);
    }
  }
  return X;
}

Mat transpose(const Mat& A) {
  Mat T(A.cols, A.rows);
  for (int i = 0; i < A.rows; ++i)
    for (int j = 0; j < A.cols; ++j) T(j, i) = A(i, j);
  return T;
}

Mat matmul(const Mat& A, const Mat& B) {
  if (A.cols != B.rows) throw std::runtime_error("matmul shape");
  Mat C(A.rows, B.cols);
  for (int i = 0; i < A.rows; ++i)
    for (int k = 0; k < A.cols; ++k) {
      const double a = A(i, k);
      if (a == 0.0) continue;
      for (int j = 0; j < B.cols; ++j) C(i, j) += a * B(k, j);
    }
  return C;
}

bool lu_inverse(const Mat& A0, Mat& Ainv, double tol) {
  const int n = A0.rows;
  Mat A = A0;
  std::vector<int> perm(n);
  double amax = 0;
  for (double v : A.a) amax = std::max(amax, std::fabs(v));
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A(i, k)) > std::fabs(A(piv, k))) piv = i;
    if (std::fabs(A(piv, k)) <= tol * amax) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A(k, j), A(piv, j));
      std::swap(perm[k], perm[piv]);
    }
    for (int i = k + 1; i < n; ++i) {
      A(i, k) /= A(k, k);
      const double l = A(i, k);
      if (l != 0.0)
        for (int j = k + 1; j < n; ++j) A(i, j) -= l * A(k, j);
    }
  }
  // solve A X = I column by column: P A = L U  ->  x = U^-1 L^-1 P e_c
  Ainv = Mat(n, n);
  Vec y(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = (perm[i] == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= A(i, k) * y[k];
      y[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < n; ++k) s -= A(i, k) * Ainv(k, c);
      Ainv(i, c) = s / A(i, i);
    }
  }
  return true;
}

// ---- geometry ------------------------------------------------------------
static const double kWmid = 0.70710678118654752440;  // 1/sqrt(2)

// Rational quadratic quarter circle: C = (N0 P0 + w N1 P1 + N2 P2) / D.
static void quarter_circle(double xi, double* C, double* dC) {
  const double b0 = (1 - xi) * (1 - xi), b1 = 2 * xi * (1 - xi), b2 = xi * xi;
  const double d0 = -2 * (1 - xi), d1 = 2 - 4 * xi, d2 = 2 * xi;
  const double D = b0 + kWmid * b1 + b2, dD = d0 + kWmid * d1 + d2;
  const double nx = b0 + kWmid * b1, ny = kWmid * b1 + b2;
  const double dnx = d0 + kWmid * d1, dny = kWmid * d1 + d2;
  C[0] = nx / D;
  C[1] = ny / D;
  dC[0] = (dnx * D - nx * dD) / (D * D);
  dC[1] = (dny * D - ny * dD) / (D * D);
}

// B-splines of degree p on span s at x and their first derivatives:
// N[r] = B_{s-p+r}(x), dN[r] = B'_{s-p+r}(x), r = 0..p.  The degree p-1 values
// on the span give the derivatives by dB_{i,p} = p (B_{i,p-1} / (t_{i+p} - t_i)
// - B_{i+1,p-1} / (t_{i+p+1} - t_{i+1})).
static void basis_with_derivative(const Vec& t, int p, int s, double x, double* N, double* dN) {
  double lower[32];
  nonzero_basis(t, p - 1, s, x, lower);      // B_{s-p+1..s, p-1}
  nonzero_basis(t, p, s, x, N);
  for (int r = 0; r <= p; ++r) {
    const int i = s - p + r;
    double d = 0.0;
    if (r >= 1) {
      const double den = t[i + p] - t[i];
      if (den > 0) d += lower[r - 1] / den;
    }
    if (r <= p - 1) {
      const double den = t[i + p + 1] - t[i + 1];
      if (den > 0) d -= lower[r] / den;
    }
    dN[r] = p * d;
  }
}

std::string NurbsVolume::check() const {
  size_t ncw = 1;
  for (int k = 0; k < 3; ++k) {
    if (p[k] < 1 || p[k] > 30) return "NURBS degree must be in 1..30";
    if (n[k] < p[k] + 1) return "NURBS needs at least degree + 1 control points per direction";
    if ((int)t[k].size() != n[k] + p[k] + 1) return "NURBS knot vector has the wrong length";
    for (size_t i = 1; i < t[k].size(); ++i)
      if (!(t[k][i] >= t[k][i - 1])) return "NURBS knots must be non-decreasing";
    for (int i = 0; i <= p[k]; ++i)
      if (t[k][i] != 0.0 || t[k][n[k] + i] != 1.0) return "NURBS knot vectors must be open on [0, 1]";
    ncw *= (size_t)n[k];
  }
  if (cw.size() != 4 * ncw) return "NURBS control net has the wrong size";
  for (size_t j = 0; j < ncw; ++j) {
    if (!(cw[4 * j + 3] > 0) || !std::isfinite(cw[4 * j + 3])) return "NURBS weights must be finite and > 0";
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(cw[4 * j + c])) return "NURBS control points must be finite";
  }
  return "";
}

Vec NurbsVolume::c0_lines(int k) const {
  Vec lines;
  const Vec& tk = t[k];
  for (size_t i = 0; i < tk.size();) {
    size_t j = i;
    while (j < tk.size() && tk[j] == tk[i]) ++j;
    if (tk[i] > tk.front() && tk[i] < tk.back() && (int)(j - i) >= p[k]) lines.push_back(tk[i]);
    i = j;
  }
  return lines;
}

void NurbsVolume::eval(const double* xh, double* x, double* dF, double* W, const char* left) const {
  double N[3][32], dN[3][32];
  int s[3];
  for (int k = 0; k < 3; ++k) {
    s[k] = find_span(t[k], p[k], xh[k], left && left[k]);
    basis_with_derivative(t[k], p[k], s[k], xh[k], N[k], dN[k]);
  }
  // homogeneous sums A = sum w P N, w = sum w N, and their derivatives
  double A[4] = {0, 0, 0, 0}, dA[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  for (int c = 0; c <= p[2]; ++c) {
    const int j3 = s[2] - p[2] + c;
    for (int b = 0; b <= p[1]; ++b) {
      const int j2 = s[1] - p[1] + b;
      const double v23 = N[1][b] * N[2][c], d2 = dN[1][b] * N[2][c], d3 = N[1][b] * dN[2][c];
      for (int a = 0; a <= p[0]; ++a) {
        const int j1 = s[0] - p[0] + a;
        const double* q = &cw[4 * ((size_t)j1 + (size_t)n[0] * (j2 + (size_t)n[1] * j3))];
        const double v = N[0][a] * v23, v1 = dN[0][a] * v23, v2 = N[0][a] * d2, v3 = N[0][a] * d3;
        for (int m = 0; m < 4; ++m) {
          A[m] += v * q[m];
          dA[0][m] += v1 * q[m];
          dA[1][m] += v2 * q[m];
          dA[2][m] += v3 * q[m];
        }
      }
    }
  }
  const double w = A[3];
  for (int c = 0; c < 3; ++c) x[c] = A[c] / w;
  if (dF)
    for (int c = 0; c < 3; ++c)
      for (int k = 0; k < 3; ++k) dF[3 * c + k] = (dA[k][c] - x[c] * dA[k][3]) / w;
  if (W) *W = w;
}

Vec Geometry::c0_lines(int k) const { return domain == 2 ? nurbs.c0_lines(k) : Vec(); }

void Geometry::eval(const double* xh, double* x, double* detJ, double* W, const char* left) const {
  if (W) *W = 1.0;
  if (domain == 0) {
    for (int k = 0; k < 3; ++k) x[k] = lo[k] + (hi[k] - lo[k]) * xh[k];
    if (detJ) *detJ = std::fabs((hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]));
  } else if (domain == 1) {
    double C[2], dC[2];
    quarter_circle(xh[0], C, dC);
    const double r = r0 + (r1 - r0) * xh[1];
    x[0] = r * C[0];
    x[1] = r * C[1];
    x[2] = height * xh[2];
    // columns dF/dxi = r C', dF/deta = (r1-r0) C, dF/dzeta = height e_z
    if (detJ) *detJ = std::fabs(r * (r1 - r0) * height * (C[0] * dC[1] - C[1] * dC[0]));
  } else {
    double F[9];
    nurbs.eval(xh, x, detJ ? F : nullptr, W, left);
    if (detJ)
      *detJ = std::fabs(F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
                        F[2] * (F[3] * F[7] - F[4] * F[6]));
  }
}

void Geometry::center(double* c) const {
  if (domain == 0) {
    for (int k = 0; k < 3; ++k) c[k] = 0.5 * (lo[k] + hi[k]);
  } else if (domain == 1) {
    // the quarter annulus lies in [0, r1] x [0, r1] x [0, height]
    c[0] = c[1] = 0.5 * r1;
    c[2] = 0.5 * height;
  } else {
    double lo3[3] = {INFINITY, INFINITY, INFINITY}, hi3[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (size_t j = 0; j + 3 < nurbs.cw.size(); j += 4)
      for (int k = 0; k < 3; ++k) {
        const double v = nurbs.cw[j + k] / nurbs.cw[j + 3];
        lo3[k] = std::min(lo3[k], v);
        hi3[k] = std::max(hi3[k], v);
      }
    for (int k = 0; k < 3; ++k) c[k] = 0.5 * (lo3[k] + hi3[k]);
  }
}

double Geometry::weight1d(int k, double t) const {
  if (domain == 1 && k == 0) return (1 - t) * (1 - t) + kWmid * 2 * t * (1 - t) + t * t;
  return 1.0;
}

}  // namespace ka

namespace ka {

bool trial_matrix_1d(const Geometry& geo, bool dir_weights, const Vec& t, int p, int k, const Vec& x, Mat& out) {
  out = bspline_matrix(t, p, x);
  if (!dir_weights) return true;
  const Vec g = greville(t, p);
  Mat Bg = bspline_matrix(t, p, g), Bgi;
  if (!lu_inverse(Bg, Bgi)) return false;
  Vec wf(g.size()), w(g.size(), 0.0);
  for (size_t i = 0; i < g.size(); ++i) wf[i] = geo.weight1d(k, g[i]);
  for (size_t i = 0; i < g.size(); ++i)
    for (size_t j = 0; j < g.size(); ++j) w[i] += Bgi(i, j) * wf[j];
  for (int a = 0; a < out.rows; ++a) {
    double den = 0;
    for (int j = 0; j < out.cols; ++j) den += w[j] * out(a, j);
    for (int j = 0; j < out.cols; ++j) out(a, j) = w[j] * out(a, j) / den;
  }
  return true;
}

}  // namespace ka
