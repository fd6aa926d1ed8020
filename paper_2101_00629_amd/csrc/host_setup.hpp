// Host-side FP64 set-up of the univariate spline factors and point sets.
//
// Everything here runs once per problem in ka_setup: knot vectors, B-spline
// evaluation, Greville abscissae, Gauss-Legendre rules, the univariate
// matrices of the Kronecker factorisations (paper Sec. 3.1 and 3.2) and their
// dense factorisations, and the closed-form geometry maps.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace ka {

using Vec = std::vector<double>;

// Row-major dense matrix.
struct Mat {
  int rows = 0, cols = 0;
  Vec a;
  Mat() = default;
  Mat(int r, int c) : rows(r), cols(c), a((size_t)r * c, 0.0) {}
  double& operator()(int i, int j) { return a[(size_t)i * cols + j]; }
  double operator()(int i, int j) const { return a[(size_t)i * cols + j]; }
};

// Open uniform knot vector on [0,1]: p+1 end knots, interior breakpoints of
// multiplicity `mult` (continuity C^{p-mult}).
Vec open_knots(int p, int nel, int mult);
int num_basis(const Vec& t, int p);

// Values of all num_basis B-splines at x (dense row of length n).
void bspline_row(const Vec& t, int p, double x, double* row);
// n x len(x) evaluation matrix B[a][c] = B_c(x_a).
Mat bspline_matrix(const Vec& t, int p, const Vec& x);

Vec greville(const Vec& t, int p);

// q-point Gauss-Legendre rule on [a,b].
void gauss_legendre(int q, double a, double b, Vec& x, Vec& w);
// Gauss points of every element (non-empty knot span), element-major.
void element_gauss(const Vec& t, int q, Vec& x, Vec& w);

// integral of B^a_i B^b_j over [0,1] (shared breakpoints).
Mat mass_matrix(const Vec& ta, int pa, const Vec& tb, int pb);

// Dense FP64 factorisations.
bool cholesky_lower(const Mat& A, Mat& L);             // A = L L^T
Mat lower_inverse(const Mat& L);                        // L^-1 (lower triangular)
Mat transpose(const Mat& A);
Mat matmul(const Mat& A, const Mat& B);
// Inverse through LU with partial pivoting (P A = L U); returns false if a
// pivot falls below tol * max|A|.
bool lu_inverse(const Mat& A, Mat& Ainv, double tol = 1e-13);

// Geometry: parametric point -> physical point, |det DF|.
struct Geometry {
  int domain = 0;              // 0 box, 1 quarter annulus
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  double r0 = 1, r1 = 2, height = 1;
  void map(const double* xh, double* x) const;
  double detJ(const double* xh) const;
  double volume() const;
  // midpoint of the axis-aligned bounding box of the mapped domain
  void center(double* c) const;
  // NURBS weight function of parametric direction k (1 for B-spline directions).
  double weight1d(int k, double t) const;
};

}  // namespace ka
