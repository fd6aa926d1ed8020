// C ABI entry points: problem set-up, the matrix-free operators, the Kronecker
// solves, the raw kernel product and the block eigensolver driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_setup.hpp"
#include "ka_internal.hpp"

namespace ka {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

const char* last_error_cstr() { return g_last_error.c_str(); }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(KA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

float kernel_coord_scale(int kernel, double ell) {
  if (std::isinf(ell)) return 0.0f;
  const double log2e = 1.4426950408889634074;
  return kernel == KA_GAUSSIAN ? (float)(std::sqrt(log2e) / ell) : (float)(log2e / ell);
}

static double coord_scale64(int kernel, double ell) {
  if (std::isinf(ell)) return 0.0;
  const double log2e = 1.4426950408889634074;
  return kernel == KA_GAUSSIAN ? std::sqrt(log2e) / ell : log2e / ell;
}

// ---------------------------------------------------------------------------
// sizes
// ---------------------------------------------------------------------------
struct Sizes {
  int n[3], nt[3], nq[3];
  int64_t N, Nt, Nq, n_rows, n_cols;
  int mult[3];
  Vec tsol[3], tint[3];   // knot vectors of the solution and (IBQ) interpolation spaces
};

// Geometry data of a KA_NURBS description; empty string, or why it is invalid.
static std::string nurbs_from_desc(const ka_desc* d, NurbsVolume& nv) {
  if (!d->geo_knots || !d->geo_ctrl) return "KA_NURBS needs geo_knots and geo_ctrl";
  size_t off = 0, ncw = 1;
  for (int k = 0; k < 3; ++k) {
    nv.p[k] = d->geo_degree[k];
    nv.n[k] = d->geo_nctrl[k];
    if (nv.p[k] < 1 || nv.p[k] > 30 || nv.n[k] < nv.p[k] + 1 || nv.n[k] > 100000)
      return "KA_NURBS needs geo_degree in 1..30 and geo_degree < geo_nctrl <= 100000";
    const size_t len = (size_t)nv.n[k] + nv.p[k] + 1;
    nv.t[k].assign(d->geo_knots + off, d->geo_knots + off + len);
    off += len;
    ncw *= (size_t)nv.n[k];
  }
  if (ncw > ((size_t)1 << 26)) return "KA_NURBS control net too large";
  // homogeneous coordinates (w x, w y, w z, w)
  nv.cw.resize(4 * ncw);
  for (size_t j = 0; j < ncw; ++j) {
    const double w = d->geo_ctrl[4 * j + 3];
    for (int c = 0; c < 3; ++c) nv.cw[4 * j + c] = w * d->geo_ctrl[4 * j + c];
    nv.cw[4 * j + 3] = w;
  }
  return nv.check();
}

static int check_desc(const ka_desc* d, Sizes& z) {
  if (!d) return fail(KA_ERR_ARG, "desc is NULL");
  if (d->method != KA_GALERKIN_IBQ && d->method != KA_COLLOCATION && d->method != KA_GALERKIN_GAUSS)
    return fail(KA_ERR_ARG, "bad method");
  if (d->domain != KA_BOX && d->domain != KA_QUARTER_ANNULUS && d->domain != KA_NURBS)
    return fail(KA_ERR_ARG, "bad domain");
  if (d->kernel != KA_GAUSSIAN && d->kernel != KA_EXP_L1) return fail(KA_ERR_ARG, "bad kernel");
  if (d->precision != KA_FP32 && d->precision != KA_BF16X3) return fail(KA_ERR_ARG, "bad precision");
  if (!(d->ell > 0)) return fail(KA_ERR_ARG, "ell must be > 0");
  if (std::isinf(d->ell) && d->kernel != KA_GAUSSIAN) return fail(KA_ERR_ARG, "ell = inf needs the Gaussian kernel");
  if (!(d->sigma > 0) || std::isinf(d->sigma)) return fail(KA_ERR_ARG, "sigma must be finite and > 0");
  if (d->block != 16 && d->block != 32 && d->block != 64) return fail(KA_ERR_ARG, "block must be 16, 32 or 64");
  if (d->domain == KA_BOX) {
    for (int k = 0; k < 3; ++k)
      if (!(d->hi[k] > d->lo[k])) return fail(KA_ERR_ARG, "box needs hi > lo");
  }
  // The geometry's C^0 lines (Sec. 4.1): the solution space is C^0 there and
  // the IBQ interpolation space C^-1 (a broken space).
  Vec lines[3];
  if (d->domain == KA_NURBS) {
    NurbsVolume nv;
    const std::string why = nurbs_from_desc(d, nv);
    if (!why.empty()) return fail(KA_ERR_ARG, why);
    for (int k = 0; k < 3; ++k) lines[k] = nv.c0_lines(k);
  } else if (d->domain == KA_QUARTER_ANNULUS) {
    if (!(d->r1 > d->r0 && d->r0 > 0 && d->height > 0)) return fail(KA_ERR_ARG, "annulus needs 0 < r0 < r1, height > 0");
  }
  z.N = z.Nt = z.Nq = 1;
  for (int k = 0; k < 3; ++k) {
    const int p = d->degree[k], e = d->nel[k];
    if (p < 1 || p > 8) return fail(KA_ERR_ARG, "degree must be in 1..8");
    if (e < 1 || e > 4096) return fail(KA_ERR_ARG, "nel must be in 1..4096");
    if (lines[k].size() > 4096) return fail(KA_ERR_ARG, "too many C0 lines in the geometry");
    int mult = 1;
    if (d->method == KA_GALERKIN_IBQ) {
      if (d->interp_cont < 0) mult = (d->kernel == KA_EXP_L1) ? p : 1;
      else if (d->interp_cont <= p - 1) mult = p - d->interp_cont;
      else return fail(KA_ERR_ARG, "interp_cont must be -1 or 0..p-1");
    }
    z.mult[k] = mult;
    z.tsol[k] = analysis_knots(p, e, 1, lines[k], p);
    z.tint[k] = analysis_knots(p, e, mult, lines[k], p + 1);
    z.n[k] = num_basis(z.tsol[k], p);
    z.nt[k] = num_basis(z.tint[k], p);
    int elems = 0;
    for (size_t i = 0; i + 1 < z.tsol[k].size(); ++i) elems += z.tsol[k][i + 1] > z.tsol[k][i];
    const int q = d->nq > 0 ? d->nq : p + 1;
    if (q > 16) return fail(KA_ERR_ARG, "nq must be <= 16");
    z.nq[k] = q * elems;
    z.N *= z.n[k];
    z.Nt *= z.nt[k];
    z.Nq *= z.nq[k];
  }
  if (d->method == KA_GALERKIN_IBQ) {
    z.Nq = 0;
    z.n_rows = z.n_cols = z.Nt;
  } else if (d->method == KA_GALERKIN_GAUSS) {
    z.Nt = 0;
    z.n_rows = z.n_cols = z.Nq;
  } else {
    z.Nt = 0;
    z.n_rows = z.N;
    z.n_cols = z.Nq;
  }
  if (z.N > (int64_t)1 << 30) return fail(KA_ERR_ARG, "problem too large");
  return KA_OK;
}

static size_t align_up(size_t x) { return (x + 255) / 256 * 256; }
// bytes one problem allocation takes (an empty buffer still takes 256)
static size_t block_bytes(size_t x) { return align_up(x ? x : 256); }

// Largest point count of any intermediate tensor of the Kronecker transfers
// (forward n -> m direction by direction, and back): sizes the FP32 buffers.
static int64_t transfer_points(const ka_desc* d, const Sizes& z) {
  const int* m = d->method == KA_GALERKIN_IBQ ? z.nt : z.nq;   // Gauss Galerkin and collocation: quadrature points
  const int64_t n0 = z.n[0], n1 = z.n[1], n2 = z.n[2], m0 = m[0], m1 = m[1], m2 = m[2];
  int64_t big = n0 * n1 * n2;
  for (int64_t v : {m0 * n1 * n2, m0 * m1 * n2, m0 * m1 * m2, n0 * m1 * m2, n0 * n1 * m2}) big = std::max(big, v);
  return big;
}

static size_t setup_bytes(const ka_desc* d, const Sizes& z) {
  const int b = d->block;
  size_t s = 0;
  for (int k = 0; k < 3; ++k) {
    s += 4 * block_bytes((size_t)z.n[k] * z.n[k] * 8);          // LinvT, Linv, Zinv, Z_k
    const int mk = d->method == KA_GALERKIN_IBQ ? z.nt[k] : z.nq[k];
    s += 2 * block_bytes((size_t)mk * z.n[k] * 4);               // T, TT
  }
  s += block_bytes((size_t)z.n_rows * 16) + block_bytes((size_t)z.n_cols * 16);
  s += block_bytes((size_t)z.n_rows * 4) + block_bytes((size_t)z.n_cols * 4);
  s += 2 * block_bytes((size_t)z.N * b * 8);
  s += 2 * block_bytes((size_t)transfer_points(d, z) * b * 4);
  s += block_bytes(gamma_plan(z.n_rows, z.n_cols, b, d->precision).work_bytes);
  if (d->domain == KA_NURBS && d->method == KA_COLLOCATION) s += block_bytes((size_t)z.n_rows * 8);   // W(g), FP64
  return s;
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
void* problem_alloc(Problem* P, size_t bytes) {
  bytes = block_bytes(bytes);
  void* p = nullptr;
  if (P->region.base) {
    if (P->region.used + bytes > P->region.size) return nullptr;
    p = P->region.base + P->region.used;
    P->region.used += bytes;
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    P->allocs.push_back({p, bytes});
  }
  P->device_bytes += bytes;
  return p;
}

static void* dev_alloc(Problem* P, size_t bytes, bool& ok) {
  void* p = ok ? problem_alloc(P, bytes) : nullptr;
  if (!p) ok = false;
  return p;
}

template <typename T>
static T* upload(Problem* P, const std::vector<T>& v, bool& ok) {
  T* p = (T*)dev_alloc(P, v.size() * sizeof(T), ok);
  if (ok && !v.empty()) ok = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
  return p;
}

static std::vector<double> to_vec(const Mat& m) { return m.a; }
static std::vector<float> to_vec32(const Mat& m) { return std::vector<float>(m.a.begin(), m.a.end()); }

static void free_problem(Problem* P) {
  if (!P) return;
  for (auto& b : P->allocs) (void)hipFree(b.p);
  if (P->eig_buf && !P->region.base) (void)hipFree(P->eig_buf);
  if (P->kl_buf) (void)hipFree(P->kl_buf);
  for (auto e : P->ev_start) (void)hipEventDestroy(e);
  for (auto e : P->ev_stop) (void)hipEventDestroy(e);
  delete P;
}

static int setup_impl(const ka_desc* d, hipStream_t stream, Problem** out, const Region* region) {
  Sizes z;
  int rc = check_desc(d, z);
  if (rc) return rc;
  Problem* P = new Problem();
  if (region) P->region = *region;
  P->d = *d;
  P->stream = stream;
  (void)hipGetDevice(&P->device);
  P->b = d->block;
  P->N = (int)z.N;
  P->Nt = (int)z.Nt;
  P->Nq = z.Nq;
  for (int k = 0; k < 3; ++k) {
    P->n[k] = z.n[k];
    P->nt[k] = z.nt[k];
    P->nq[k] = z.nq[k];
  }
  P->n_rows = z.n_rows;
  P->n_cols = z.n_cols;
  P->out_scale = (float)(d->sigma * d->sigma);
  P->coord_scale = 1.0f;   // coordinates are prescaled in FP64 below
  Geometry& geo = P->geo;   // kept: K-L sampling evaluates the trial space at new points
  geo.domain = d->domain;
  for (int k = 0; k < 3; ++k) {
    geo.lo[k] = d->lo[k];
    geo.hi[k] = d->hi[k];
  }
  geo.r0 = d->r0;
  geo.r1 = d->r1;
  geo.height = d->height;
  if (d->domain == KA_NURBS) (void)nurbs_from_desc(d, geo.nurbs);   // validated in check_desc
  // the caller's geometry arrays are not kept
  P->d.geo_knots = nullptr;
  P->d.geo_ctrl = nullptr;
  const double cs = coord_scale64(d->kernel, d->ell);
  // The kernel depends on differences only: coordinates are centred on the
  // domain before rounding to FP32, which halves their absolute rounding error.
  double ctr[3];
  geo.center(ctr);
  bool ok = true;

  // univariate factors
  std::vector<Vec> pts1d(3);      // Galerkin: interpolation Greville points; collocation: Greville points
  std::vector<Vec> q1d(3), w1d(3);
  std::vector<std::vector<char>> left1d(3);   // IBQ: interpolation points taken from the left
  for (int k = 0; k < 3; ++k) {
    const int p = d->degree[k];
    const Vec& t = z.tsol[k];
    P->tsol[k] = t;
    if (d->method == KA_GALERKIN_GAUSS) {
      // standard Galerkin (Sec. 3.1): basis values at the element Gauss points
      Mat Zk = mass_matrix(t, p, t, p), Lk;
      if (!cholesky_lower(Zk, Lk)) {
        free_problem(P);
        return fail(KA_ERR_SINGULAR, "mass matrix is not SPD");
      }
      const Mat Li = lower_inverse(Lk);
      const Mat LiT = transpose(Li);
      P->Linv[k] = upload(P, to_vec(Li), ok);
      P->LinvT[k] = upload(P, to_vec(LiT), ok);
      P->Zinv[k] = upload(P, to_vec(matmul(LiT, Li)), ok);
      P->ZinvT[k] = P->Zinv[k];   // the mass matrix is symmetric
      P->Zk[k] = upload(P, to_vec(Zk), ok);   // mass matrix: exact L2 norms of eigenfunctions
      Vec xq, wq;
      element_gauss(t, d->nq > 0 ? d->nq : p + 1, xq, wq);
      const Mat Rq = bspline_matrix(t, p, xq);                 // nq x n
      P->T[k] = upload(P, to_vec32(Rq), ok);
      P->TT[k] = upload(P, to_vec32(transpose(Rq)), ok);
      q1d[k] = xq;
      w1d[k] = wq;
    } else if (d->method == KA_GALERKIN_IBQ) {
      Mat Zk = mass_matrix(t, p, t, p), Lk;
      if (!cholesky_lower(Zk, Lk)) {
        free_problem(P);
        return fail(KA_ERR_SINGULAR, "mass matrix is not SPD");
      }
      const Mat Li = lower_inverse(Lk);
      const Mat LiT = transpose(Li);
      P->Linv[k] = upload(P, to_vec(Li), ok);
      P->LinvT[k] = upload(P, to_vec(LiT), ok);
      P->Zinv[k] = upload(P, to_vec(matmul(LiT, Li)), ok);
      P->ZinvT[k] = P->Zinv[k];   // the mass matrix is symmetric
      P->Zk[k] = upload(P, to_vec(Zk), ok);   // mass matrix: exact L2 norms of eigenfunctions
      const Vec& ti = z.tint[k];
      const Vec g = greville(ti, p);
      left1d[k] = greville_left(ti, p);                      // one-sided at C^-1 knots
      const Mat Mk = mass_matrix(ti, p, t, p);               // nt x n
      const Mat Bt = bspline_matrix(ti, p, g, &left1d[k]);   // nt x nt, rows are points
      Mat Bti;
      if (!lu_inverse(Bt, Bti)) {
        free_problem(P);
        return fail(KA_ERR_SINGULAR, "interpolation collocation matrix is singular");
      }
      const Mat Tk = matmul(transpose(Bti), Mk);             // B~^-T M
      P->T[k] = upload(P, to_vec32(Tk), ok);
      P->TT[k] = upload(P, to_vec32(transpose(Tk)), ok);
      pts1d[k] = g;
    } else {
      const Vec g = greville(t, p);
      Vec xq, wq;
      element_gauss(t, d->nq > 0 ? d->nq : p + 1, xq, wq);
      // NURBS functions of the direction (weights interpolating its weight function)
      Mat Rq, Zc;
      if (!trial_matrix_1d(geo, true, t, p, k, xq, Rq) || !trial_matrix_1d(geo, true, t, p, k, g, Zc)) {
        free_problem(P);
        return fail(KA_ERR_SINGULAR, "Greville collocation matrix is singular");
      }
      Mat Zci;
      if (!lu_inverse(Zc, Zci)) {
        free_problem(P);
        return fail(KA_ERR_SINGULAR, "collocation matrix Z_k is singular");
      }
      P->Zinv[k] = upload(P, to_vec(Zci), ok);
      P->ZinvT[k] = upload(P, to_vec(transpose(Zci)), ok);
      P->T[k] = upload(P, to_vec32(Rq), ok);
      P->TT[k] = upload(P, to_vec32(transpose(Rq)), ok);
      pts1d[k] = g;
      q1d[k] = xq;
      w1d[k] = wq;
    }
  }
  // point sets
  // mapped points (centred, prescaled FP32), optionally |det DF| and the
  // NURBS weight function W at the tensor grid g[0] x g[1] x g[2]
  // (`left`: per direction, points evaluated as limits from the left)
  auto tensor_points = [&](const std::vector<Vec>& g, std::vector<float>& xyz, std::vector<double>* detJ,
                           std::vector<double>* W = nullptr, const std::vector<std::vector<char>>* left = nullptr) {
    const int64_t n1 = g[0].size(), n2 = g[1].size(), n3 = g[2].size();
    xyz.assign((size_t)n1 * n2 * n3 * 4, 0.f);
    if (detJ) detJ->assign((size_t)n1 * n2 * n3, 0.0);
    if (W) W->assign((size_t)n1 * n2 * n3, 1.0);
    for (int64_t a3 = 0; a3 < n3; ++a3)
      for (int64_t a2 = 0; a2 < n2; ++a2)
        for (int64_t a1 = 0; a1 < n1; ++a1) {
          const int64_t i = a1 + n1 * (a2 + n2 * a3);
          const double xh[3] = {g[0][a1], g[1][a2], g[2][a3]};
          char side[3] = {0, 0, 0};
          if (left)
            for (int k = 0; k < 3; ++k) {
              const auto& lk = (*left)[k];
              const int64_t a = k == 0 ? a1 : (k == 1 ? a2 : a3);
              side[k] = lk.empty() ? 0 : lk[a];
            }
          double x[3];
          geo.eval(xh, x, detJ ? &(*detJ)[i] : nullptr, W ? &(*W)[i] : nullptr, side);
          for (int c = 0; c < 3; ++c) xyz[i * 4 + c] = (float)((x[c] - ctr[c]) * cs);
        }
  };
  if (d->method == KA_GALERKIN_IBQ) {
    std::vector<float> xyz;
    std::vector<double> dj;
    tensor_points(pts1d, xyz, &dj, nullptr, &left1d);   // |det DF| one-sided where it jumps
    std::vector<float> J(dj.size());
    for (size_t i = 0; i < dj.size(); ++i) J[i] = (float)std::sqrt(dj[i]);
    P->rows = upload(P, xyz, ok);
    P->cols = P->rows;
    P->rscale = upload(P, J, ok);
    P->cscale = P->rscale;
  } else if (d->method == KA_GALERKIN_GAUSS) {
    // trial space B_i / sqrt|det DF| (as for IBQ): both sides of Gamma carry
    // the quadrature weight times sqrt|det DF|
    std::vector<float> xyz;
    std::vector<double> dj;
    tensor_points(q1d, xyz, &dj);
    std::vector<float> ws(dj.size());
    const int64_t m1 = q1d[0].size(), m2 = q1d[1].size();
    for (size_t i = 0; i < dj.size(); ++i) {
      const int64_t a1 = i % m1, a2 = (i / m1) % m2, a3 = i / (m1 * m2);
      ws[i] = (float)(std::sqrt(dj[i]) * w1d[0][a1] * w1d[1][a2] * w1d[2][a3]);
    }
    P->rows = upload(P, xyz, ok);
    P->cols = P->rows;
    P->rscale = upload(P, ws, ok);
    P->cscale = P->rscale;
  } else {
    // General NURBS volume: trial functions B_j / W (W the geometry's weight
    // function, B_j the tensor B-splines of the univariate factors above).
    // Then R_q = diag(1/W(q)) (R_q,3 x R_q,2 x R_q,1) and Z = diag(1/W(g))
    // (Z_3 x Z_2 x Z_1): 1/W(q) joins |det DF| W on the columns, and
    // Z^-1 = (Z_3^-1 x Z_2^-1 x Z_1^-1) diag(W(g)), whose diagonal is the row
    // scale of the kernel product.
    std::vector<float> xr, xq;
    std::vector<double> wg, wq;
    tensor_points(pts1d, xr, nullptr, &wg);
    std::vector<double> dj;
    tensor_points(q1d, xq, &dj, &wq);
    std::vector<float> jw(dj.size());
    const int64_t m1 = q1d[0].size(), m2 = q1d[1].size();
    for (size_t i = 0; i < dj.size(); ++i) {
      const int64_t a1 = i % m1, a2 = (i / m1) % m2, a3 = i / (m1 * m2);
      jw[i] = (float)(dj[i] * w1d[0][a1] * w1d[1][a2] * w1d[2][a3] / wq[i]);
    }
    P->rows = upload(P, xr, ok);
    P->cols = upload(P, xq, ok);
    P->rscale = nullptr;
    if (d->domain == KA_NURBS) {
      P->rscale = upload(P, std::vector<float>(wg.begin(), wg.end()), ok);
      P->wrow64 = upload(P, wg, ok);
    }
    P->cscale = upload(P, jw, ok);
  }
  const int b = P->b;
  P->w64a = (double*)dev_alloc(P, (size_t)P->N * b * 8, ok);
  P->w64b = (double*)dev_alloc(P, (size_t)P->N * b * 8, ok);
  const int64_t big = transfer_points(d, z);
  P->w32a = (float*)dev_alloc(P, (size_t)big * b * 4, ok);
  P->w32b = (float*)dev_alloc(P, (size_t)big * b * 4, ok);
  const GammaPlan gp = gamma_plan(P->n_rows, P->n_cols, b, d->precision);
  P->gpart_bytes = gp.work_bytes;
  P->gpart = (float*)dev_alloc(P, gp.work_bytes, ok);
  if (!ok) {
    free_problem(P);
    return fail(KA_ERR_OOM, "device allocation failed in ka_setup");
  }
  if (fill_zero_f32(P->w32a, big * b, stream) != hipSuccess || fill_zero_f32(P->w32b, big * b, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    free_problem(P);
    return fail(KA_ERR_HIP, "workspace initialisation failed");
  }
  *out = P;
  return KA_OK;
}

// ---------------------------------------------------------------------------
// operator pieces
// ---------------------------------------------------------------------------
static ModeArgs mode_args(const void* in, int in_layout, int64_t in_ld, void* out, int out_layout, int64_t out_ld,
                          const int dims[3], int mode, int m, const void* mat, const void* matT, int nv,
                          const float* scale) {
  ModeArgs a;
  a.in = in;
  a.in_layout = in_layout;
  a.in_ld = in_ld;
  a.out = out;
  a.out_layout = out_layout;
  a.out_ld = out_ld;
  for (int k = 0; k < 3; ++k) a.n_in[k] = dims[k];
  a.mode = mode;
  a.m = m;
  a.mat = mat;
  a.matT = matT;
  a.nv = nv;
  a.out_scale = scale;
  return a;
}

int gamma_step(Problem* P, const float* Y, float* Z, hipStream_t s) {
  GammaLaunch g;
  g.xr = P->rows;
  g.xr_stride = 4;
  g.rs = P->rscale;
  g.nr = P->n_rows;
  g.xc = P->cols;
  g.xc_stride = 4;
  g.nc = P->n_cols;
  g.Y = Y;
  g.Z = Z;
  g.partial = P->gpart;
  g.ys = nullptr;   // launch_gamma places it in the scratch
  g.coord_scale = P->coord_scale;
  g.out_scale = P->out_scale;
  g.nsplit = 1;
  g.cols_per_split = 0;
  g.row_blocks = 0;
  g.xcd_splits = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (P->profile) {
    if (P->prof_launches < (int)P->ev_start.size()) {
      e0 = P->ev_start[P->prof_launches];
      e1 = P->ev_stop[P->prof_launches];
    } else {
      HIP_TRY(hipEventCreate(&e0));
      HIP_TRY(hipEventCreate(&e1));
      P->ev_start.push_back(e0);
      P->ev_stop.push_back(e1);
    }
    HIP_TRY(hipEventRecord(e0, s));
  }
  HIP_TRY(launch_gamma(g, P->d.kernel, P->b, P->d.precision, s));
  const double pairs = (double)P->n_rows * (double)P->n_cols;
  P->pairs_total += pairs;
  if (P->profile) {
    HIP_TRY(hipEventRecord(e1, s));
    P->prof_launches++;
    P->prof_pairs += pairs;
  }
  return KA_OK;
}

// Three FP64 mode products with per-direction matrices mats[k] (n_k x n_k) on
// a point-major block (point stride b) in `src`, through `other`; the result
// is left in `other`.
static int kron64_pt(Problem* P, double* const mats[3], double* const matsT[3], double* src, double* other, int nv,
                     hipStream_t s) {
  const int* n = P->n;
  const int b = P->b;
  HIP_TRY(launch_mode_f64(mode_args(src, LAYOUT_PT, b, other, LAYOUT_PT, b, n, 0, n[0], mats[0], matsT[0], nv, nullptr), s));
  HIP_TRY(launch_mode_f64(mode_args(other, LAYOUT_PT, b, src, LAYOUT_PT, b, n, 1, n[1], mats[1], matsT[1], nv, nullptr), s));
  HIP_TRY(launch_mode_f64(mode_args(src, LAYOUT_PT, b, other, LAYOUT_PT, b, n, 2, n[2], mats[2], matsT[2], nv, nullptr), s));
  return KA_OK;
}

// Point-major FP64 block `src` (point stride b) -> Galerkin: J B~^-T M X ;
// collocation: JW R_q X.  Output: point-major FP32 in w32b (point stride b).
static int forward_transfer(Problem* P, const double* src, int nv, hipStream_t s) {
  const int b = P->b;
  const int* n = P->n;
  const int* m = P->d.method == KA_GALERKIN_IBQ ? P->nt : P->nq;
  int d0[3] = {n[0], n[1], n[2]};
  HIP_TRY(launch_mode_f64_to_f32(mode_args(src, LAYOUT_PT, b, P->w32b, LAYOUT_PT, b, d0, 0, m[0], P->T[0], P->TT[0], nv, nullptr), s));
  int d1[3] = {m[0], n[1], n[2]};
  HIP_TRY(launch_mode_f32(mode_args(P->w32b, LAYOUT_PT, b, P->w32a, LAYOUT_PT, b, d1, 1, m[1], P->T[1], P->TT[1], nv, nullptr), s));
  int d2[3] = {m[0], m[1], n[2]};
  HIP_TRY(launch_mode_f32(mode_args(P->w32a, LAYOUT_PT, b, P->w32b, LAYOUT_PT, b, d2, 2, m[2], P->T[2], P->TT[2], nv, P->cscale), s));
  return KA_OK;   // result in w32b
}

// Operator steps before the kernel product: X (FP64, column layout) ->
// kernel-product input in w32b (point-major FP32, stride b).
//   Galerkin: [L^-T if A'], then B~^-T M per direction with J on the last store
//   (nine-step algorithm, steps 1-4).  Collocation: R_q per direction with
//   J W on the last store (Algorithm 1, steps 1-2).
int apply_pre(Problem* P, int form, const double* X, int64_t ldx, int nv, hipStream_t s) {
  const int b = P->b;
  HIP_TRY(col64_to_pt64(X, ldx, P->w64a, b, P->N, nv, s));
  double* src = P->w64a;
  if (P->d.method != KA_COLLOCATION && form == KA_APRIME) {
    if (int rc = kron64_pt(P, P->LinvT, P->Linv, P->w64a, P->w64b, nv, s)) return rc;
    src = P->w64b;
  }
  return forward_transfer(P, src, nv, s);
}

// Operator steps after the kernel product: w32a (point-major FP32) -> Y.
//   Galerkin: M^T B~^-1 per direction, [L^-1 if A'] (steps 7-9; step 6 is
//   folded into the product's store).  Collocation: [Z^-1 if A'] (step 4).
int apply_post(Problem* P, int form, double* Y, int64_t ldy, int nv, hipStream_t s) {
  const int b = P->b;
  const int* n = P->n;
  const int64_t N = P->N;
  const int nn[3] = {n[0], n[1], n[2]};
  if (P->d.method != KA_COLLOCATION) {
    const int* m = P->d.method == KA_GALERKIN_IBQ ? P->nt : P->nq;
    int d0[3] = {m[0], m[1], m[2]};
    HIP_TRY(launch_mode_f32(mode_args(P->w32a, LAYOUT_PT, b, P->w32b, LAYOUT_PT, b, d0, 0, n[0], P->TT[0], P->T[0], nv, nullptr), s));
    int d1[3] = {n[0], m[1], m[2]};
    HIP_TRY(launch_mode_f32(mode_args(P->w32b, LAYOUT_PT, b, P->w32a, LAYOUT_PT, b, d1, 1, n[1], P->TT[1], P->T[1], nv, nullptr), s));
    int d2[3] = {n[0], n[1], m[2]};
    HIP_TRY(launch_mode_f32_to_f64(mode_args(P->w32a, LAYOUT_PT, b, P->w64b, LAYOUT_PT, b, d2, 2, n[2], P->TT[2], P->T[2], nv, nullptr), s));
    double* res = P->w64b;
    if (form == KA_APRIME) {
      if (int rc = kron64_pt(P, P->Linv, P->LinvT, P->w64b, P->w64a, nv, s)) return rc;
      res = P->w64a;
    }
    HIP_TRY(pt64_to_col64(res, b, Y, ldy, N, nv, s));
    return KA_OK;
  }
  if (form == KA_APRIME) {
    HIP_TRY(launch_mode_f32in_f64(mode_args(P->w32a, LAYOUT_PT, b, P->w64a, LAYOUT_PT, b, nn, 0, n[0], P->Zinv[0], P->ZinvT[0], nv, nullptr), s));
    HIP_TRY(launch_mode_f64(mode_args(P->w64a, LAYOUT_PT, b, P->w64b, LAYOUT_PT, b, nn, 1, n[1], P->Zinv[1], P->ZinvT[1], nv, nullptr), s));
    HIP_TRY(launch_mode_f64(mode_args(P->w64b, LAYOUT_PT, b, P->w64a, LAYOUT_PT, b, nn, 2, n[2], P->Zinv[2], P->ZinvT[2], nv, nullptr), s));
    HIP_TRY(pt64_to_col64(P->w64a, b, Y, ldy, N, nv, s));
  } else {
    HIP_TRY(cast_pt32_to_col64(P->w32a, b, Y, ldy, N, nv, P->wrow64, s));   // A itself: W(g) divided out
  }
  return KA_OK;
}

// The kernel-product job of one block application (input w32b, output
// w32a), for single or batched launches.
GammaLaunch gamma_job(Problem* P) {
  GammaLaunch g;
  g.xr = P->rows;
  g.xr_stride = 4;
  g.rs = P->rscale;
  g.nr = P->n_rows;
  g.xc = P->cols;
  g.xc_stride = 4;
  g.nc = P->n_cols;
  g.Y = P->w32b;
  g.Z = P->w32a;
  g.partial = P->gpart;
  g.coord_scale = P->coord_scale;
  g.out_scale = P->out_scale;
  const GammaPlan gp = gamma_plan(g.nr, g.nc, P->b, P->d.precision);
  g.nsplit = gp.nsplit;
  g.cols_per_split = gp.cols_per_split;
  g.row_blocks = gp.row_blocks;
  g.ys = gamma_ysplit_ptr(P->gpart, gp);   // batched launches run the split pre-pass themselves
  g.xcd_splits = 0;   // batched launches enumerate (row block, split) items explicitly
  return g;
}

int apply_block(Problem* P, int form, const double* X, int64_t ldx, double* Y, int64_t ldy, int nv, hipStream_t s) {
  int rc;
  if ((rc = apply_pre(P, form, X, ldx, nv, s))) return rc;
  if ((rc = gamma_step(P, P->w32b, P->w32a, s))) return rc;
  return apply_post(P, form, Y, ldy, nv, s);
}

int solve_block(Problem* P, int op, double* X, int64_t ld, int nv, hipStream_t s) {
  double* const* mats = nullptr;
  double* const* matsT = nullptr;
  if (op == KA_ZINV) {
    if (P->wrow64) HIP_TRY(scale_rows(X, P->N, nv, ld, P->wrow64, s));   // general NURBS: diag(W(g)) first
    mats = P->Zinv;
    matsT = P->ZinvT;
  } else if (P->d.method == KA_COLLOCATION) {
    return fail(KA_ERR_STATE, "L solves exist for the Galerkin methods only");
  } else if (op == KA_LINV) {
    mats = P->Linv;
    matsT = P->LinvT;
  } else if (op == KA_LTINV) {
    mats = P->LinvT;
    matsT = P->Linv;
  } else {
    return fail(KA_ERR_ARG, "bad solve op");
  }
  HIP_TRY(col64_to_pt64(X, ld, P->w64a, P->b, P->N, nv, s));
  if (int rc = kron64_pt(P, mats, matsT, P->w64a, P->w64b, nv, s)) return rc;
  HIP_TRY(pt64_to_col64(P->w64b, P->b, X, ld, P->N, nv, s));
  return KA_OK;
}

}  // namespace ka

namespace ka {
int setup_problem(const ka_desc* d, hipStream_t stream, Problem** out, const Region* region) {
  return setup_impl(d, stream, out, region);
}

int footprint(const ka_desc* d, size_t* bytes) {
  Sizes z;
  int rc = check_desc(d, z);
  if (rc) return rc;
  *bytes = setup_bytes(d, z);
  return KA_OK;
}

int desc_sizes(const ka_desc* d, int64_t* N, int64_t* Nt, int64_t* Nq) {
  Sizes z;
  int rc = check_desc(d, z);
  if (rc) return rc;
  if (N) *N = z.N;
  if (Nt) *Nt = z.Nt;
  if (Nq) *Nq = z.Nq;
  return KA_OK;
}

void destroy_problem(Problem* P) { free_problem(P); }
}  // namespace ka
