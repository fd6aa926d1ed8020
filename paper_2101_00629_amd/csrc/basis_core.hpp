// Orthonormal basis of the span of a set of vectors, from their Gram matrix,
// for the thick restart of the non-symmetric (collocation) eigensolver: the
// kept Ritz vectors S (columns of the projected space) are in general not
// orthogonal, and the restarted Krylov basis is X S W with W such that S W
// has orthonormal columns.
//
// Diagonal-pivoted Cholesky of the positive semi-definite G = S^T S: at step
// j the largest remaining diagonal entry is moved to position j (rows and
// columns swapped), R(j, j) is its square root, row j of R is the rest of
// row j divided by it, and the trailing block loses the outer product of that
// row.  The remaining diagonal entries are the squared distances of the
// remaining vectors from the span of the chosen ones, so the factorisation
// stops at the first pivot at or below cut * max_i G(i, i): the vectors from
// there on are dependent on the chosen ones to that accuracy.  With the r
// chosen pivots P^T G P = R^T R (leading r x r), and W = P[:, :r] R^-1.
// (Textbook pivoted Cholesky, e.g. Golub and Van Loan Sec. 4.2.8; the rank cut
// replaces the eigenvalue cut of a Gram eigendecomposition.)
//
// Written once over a team of threads (tid(), size(), sync(), and
// argmax(v, i): the index i of the largest v over the team, the smallest
// index among equals, -1 when no thread has one (i < 0), returned to every
// thread), so the same source runs as one
// workgroup on the device and as one thread in the host unit tests.
#pragma once
#include <math.h>
#include <stddef.h>

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

KA_HD inline size_t pchol_basis_work(int n) { return (size_t)n * n + 2 * (size_t)n; }   // doubles

// G: n x n (column-major, leading dimension ldg), symmetric positive
// semi-definite.  work: team-shared, pchol_basis_work(n) doubles (fast memory
// where it fits): the working copy, whose upper triangle becomes R and whose
// strictly lower triangle then holds R^-1 transposed, the diagonal of R^-1,
// and the pivot order.  W: n x n (leading dimension ldw): columns 0 .. r-1
// receive the basis coefficients, the others are left untouched.  Returns r
// (0 when G is zero).  Inlined, so that each caller accesses its work array
// with the instructions of that array's address space.
template <class Team>
KA_HD KA_FORCEINLINE int pchol_basis(Team& tm, const double* G, int ldg, int n, double cut, double* work, double* W, int ldw) {
  const int t = tm.tid(), NT = tm.size();
  if (n <= 0) return 0;
  double* A = work;                         // working copy; R in its upper triangle
  double* xd = A + (size_t)n * n;           // diagonal of R^-1
  int* piv = reinterpret_cast<int*>(xd + n);
#define AA(i, j) A[(size_t)(j) * n + (i)]
#define XX(i, j) ((i) == (j) ? xd[i] : A[(size_t)(i) * n + (j)])   // R^-1 (i <= j), stored transposed below
  for (size_t e = t; e < (size_t)n * n; e += NT) AA(e % n, e / n) = G[(e / n) * (size_t)ldg + e % n];
  for (int i = t; i < n; i += NT) piv[i] = i;
  tm.sync();
  int best = -1;
  double bv = -1.0;
  for (int i = t; i < n; i += NT)
    if (AA(i, i) > bv) {
      bv = AA(i, i);
      best = i;
    }
  const int i0 = tm.argmax(bv, best);
  const double dmax = i0 >= 0 ? AA(i0, i0) : 0.0;
  tm.sync();
  int r = n;
  for (int j = 0; j < n; ++j) {
    best = -1;
    bv = -1.0;
    for (int i = j + t; i < n; i += NT)
      if (AA(i, i) > bv) {
        bv = AA(i, i);
        best = i;
      }
    const int p = tm.argmax(bv, best);
    const double d = p >= 0 ? AA(p, p) : 0.0;
    if (!(d > cut * dmax) || !(d > 0.0)) {
      r = j;
      break;
    }
    tm.sync();
    if (p != j) {                                       // symmetric swap of rows and columns j and p
      for (int i = t; i < n; i += NT) {
        const double x = AA(j, i);
        AA(j, i) = AA(p, i);
        AA(p, i) = x;
      }
      tm.sync();
      for (int i = t; i < n; i += NT) {
        const double x = AA(i, j);
        AA(i, j) = AA(i, p);
        AA(i, p) = x;
      }
      if (t == 0) {
        const int x = piv[j];
        piv[j] = piv[p];
        piv[p] = x;
      }
      tm.sync();
    }
    const double rjj = sqrt(d), inv = 1.0 / rjj;
    for (int i = j + 1 + t; i < n; i += NT) AA(j, i) *= inv;   // row j of R (columns j+1 ..)
    if (t == 0) AA(j, j) = rjj;
    tm.sync();
    const int m = n - j - 1;                            // trailing block: A(i, l) -= R(j, i) R(j, l)
    for (size_t e = t; e < (size_t)m * m; e += NT) {
      const int i = j + 1 + (int)(e % m), l = j + 1 + (int)(e / m);
      AA(i, l) -= AA(j, i) * AA(j, l);
    }
    tm.sync();
  }
  tm.sync();
  // X = R^-1 row by row from the bottom: X(i, i) = 1 / R(i, i) and
  // X(i, c) = -X(i, i) * sum_{k = i+1 .. c} R(i, k) X(k, c), one thread per c.
  // (the strictly lower triangle of the working copy is free once R is done)
  for (int i = r - 1; i >= 0; --i) {
    const double d = 1.0 / AA(i, i);
    for (int c = i + t; c < r; c += NT) {
      if (c == i) {
        xd[i] = d;
      } else {
        double s = AA(i, c) * xd[c];
        for (int k = i + 1; k < c; ++k) s += AA(i, k) * A[(size_t)k * n + c];
        A[(size_t)i * n + c] = -d * s;
      }
    }
    tm.sync();
  }
  // W = P[:, :r] R^-1: row i of R^-1 lands in row piv[i] of W
  for (size_t e = t; e < (size_t)r * n; e += NT) {
    const int i = (int)(e % n), c = (int)(e / n);
    W[(size_t)c * ldw + piv[i]] = (i <= c) ? XX(i, c) : 0.0;
  }
  tm.sync();
#undef AA
#undef XX
  return r;
}

}  // namespace ka
