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
// Knot vector of an analysis space (paper Sec. 4.1): nel uniform elements
// with interior multiplicity `mult`, plus `lines` (positions where the
// geometry is only C^0) with multiplicity `line_mult` (p: C^0, p+1: C^-1),
// added to the mesh where they are not uniform breakpoints already.
Vec analysis_knots(int p, int nel, int mult, const Vec& lines, int line_mult);
int num_basis(const Vec& t, int p);

// Values of all num_basis B-splines at x (dense row of length n); `left`
// takes the limit from the left, which differs only at a knot of
// multiplicity p+1 (a broken space).
void bspline_row(const Vec& t, int p, double x, double* row, bool left = false);
// n x len(x) evaluation matrix B[a][c] = B_c(x_a), optionally one-sided per point.
Mat bspline_matrix(const Vec& t, int p, const Vec& x, const std::vector<char>* left = nullptr);

Vec greville(const Vec& t, int p);
// Greville abscissae taken as limits from the left: at a knot of
// multiplicity p+1 the last function of the left piece and the first of the
// right piece share one abscissa; each is evaluated from its own side, which
// keeps the interpolation matrix non-singular.
std::vector<char> greville_left(const Vec& t, int p);

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

// Single-patch NURBS volume (paper Sec. 3.2: the geometry is given by NURBS):
// F(xh) = sum_j w_j P_j N_j(xh) / W(xh) with W(xh) = sum_j w_j N_j(xh), N_j the
// tensor-product B-splines of the geometry's own degrees and knot vectors.
struct NurbsVolume {
  int p[3] = {0, 0, 0};
  int n[3] = {0, 0, 0};        // control points per direction
  Vec t[3];                    // open knot vectors on [0, 1]
  Vec cw;                      // homogeneous control points (w x, w y, w z, w), index j1 + n1 (j2 + n2 j3)
  // Empty string if the data describe a valid volume, else the reason.
  std::string check() const;
  // Point x, Jacobian dF[3 c + k] = d x_c / d xh_k and weight function W at
  // xh; left[k] (optional) takes direction k's limit from the left, where dF
  // jumps across a C^0 line.
  void eval(const double* xh, double* x, double* dF, double* W, const char* left = nullptr) const;
  // Interior knots of direction k repeated at least p[k] times: the map is
  // only C^0 there (for instance where two patches meet).
  Vec c0_lines(int k) const;
};

// Trial-space factor of parametric direction k at points x (rows are points):
// the degree-p B-splines on knots t, or, with dir_weights, the NURBS functions
// w_j B_j / sum_l w_l B_l whose weights interpolate the direction's weight
// function (geo.weight1d) at the Greville points.  Returns false if that
// interpolation matrix is singular.
struct Geometry;
bool trial_matrix_1d(const Geometry& geo, bool dir_weights, const Vec& t, int p, int k, const Vec& x, Mat& out);

// Geometry: parametric point -> physical point, |det DF|.
struct Geometry {
  int domain = 0;              // 0 box, 1 quarter annulus, 2 general NURBS volume
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  double r0 = 1, r1 = 2, height = 1;
  NurbsVolume nurbs;
  // Mapped point, and optionally |det DF| and the NURBS weight function W
  // (general NURBS volume; 1 for the closed-form domains).  left[k]
  // (optional) takes direction k's limit from the left at a C^0 line.
  void eval(const double* xh, double* x, double* detJ, double* W, const char* left = nullptr) const;
  // C^0 lines of parametric direction k (general NURBS volume only).
  Vec c0_lines(int k) const;
  // midpoint of the axis-aligned bounding box of the mapped domain (of the
  // control points for a NURBS volume, which contain it)
  void center(double* c) const;
  // Weight function of parametric direction k when the weights are a tensor
  // product (the quarter annulus); 1 for B-spline directions and for the
  // general NURBS volume, whose weight function enters through eval().
  double weight1d(int k, double t) const;
};

}  // namespace ka
