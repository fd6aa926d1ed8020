"""Matrix-free isogeometric collocation (paper Sec. 3.2).

The residual of the Fredholm problem is required to vanish at the Greville
abscissae g_i of the trial space (eq. colloc_residual), giving
    A_ij = integral over D of Gamma(x_i, x') R_j(x') dx',   Z_ij = R_j(g_i)
(eq. colloc_system_matrices), with x_i = F(g_i) and R_j the NURBS trial
functions of the isoparametric geometry.  A is evaluated with a tensor
Gauss-Legendre rule of nq points per element and direction:
    A = Gamma_c diag(J * W) R_q,
Gamma_c[i, k] = Gamma(x_i, F(q_k)), J_k = |det DF(q_k)|, W_k the product
Gauss weight, R_q[k, j] = R_j(q_k).

The standard form is A' = Q U^-1 L^-1 P A from the pivoted LU of Z
(eq. for A' in Sec. 3.2), applied with Algorithm 1:
    1  y  = R_q v          (interpolate at quadrature points)
    2  y' = y * J * W      (scale)
    3  z  = Gamma_c y'     (kernel rows on the fly)
    4  v' = Z^-1 z         (backsolve with the LU of Z)

NURBS weights: for the quarter annulus the rational direction has weight
function D(xi), a quadratic; its control weights w in the degree-p space are
obtained by interpolation at the Greville points (exact, as D lies in the
space), and R_j = w_j B_j / (sum_l w_l B_l).  Because the weights are a
tensor product, Z = Z_3 x Z_2 x Z_1 (remark in Sec. 3.3).

General NURBS volume (domain.rational): the weights need not be a tensor
product.  The trial space is spanned by B_j / W (W the geometry's weight
function, B_j the tensor B-splines), the span of the NURBS functions
w_j B_j / W.  The oracle assembles R_q and Z point by point and, as the paper
does when Z has no Kronecker structure, factors the full Z with a complete-
pivoting LU (P Z Q = L U) to apply Z^-1.
"""
import numpy as np
import scipy.linalg as sla

from . import splines, kernels, kron
from .geometry import make_domain, c0_lines


class _LUSolve:
    def __init__(self, A):
        self.lu = sla.lu_factor(A)     # partial (row) pivoting, LAPACK getrf
        self.n = A.shape[0]

    def __call__(self, X):
        return sla.lu_solve(self.lu, X)


def nurbs_basis_1d(knots, p, weight_fn, x):
    """R_j(x) = w_j B_j(x) / sum_l w_l B_l(x) with w interpolating weight_fn."""
    g = splines.greville(knots, p)
    w = np.linalg.solve(splines.basis_matrix(knots, p, g), weight_fn(g))
    B = splines.basis_matrix(knots, p, x)
    return B * w[None, :] / (B @ w)[:, None]


class Collocation:
    def __init__(self, domain, p, nel, kernel, ell, sigma=1.0, nq=None):
        self.domain = make_domain(domain) if isinstance(domain, str) else domain
        self.p = int(p)
        self.nel = tuple(int(e) for e in nel)
        self.kernel, self.ell, self.sigma = kernel, ell, sigma
        self.nq = int(nq or (self.p + 1))
        self.rational = bool(getattr(self.domain, "rational", False))
        self.gk, self.Rqk, self.Zk, self.xqk, self.wqk, self.knots = [], [], [], [], [], []
        for k, e in enumerate(self.nel):
            # the solution space is C^0 where the geometry is (Sec. 4.1)
            t = splines.open_knots(self.p, e, 1, lines=c0_lines(self.domain, k), line_mult=self.p)
            self.knots.append(t)
            g = splines.greville(t, self.p)
            xq, wq = splines.element_quadrature(t, self.nq)
            self.gk.append(g)
            self.xqk.append(xq)
            self.wqk.append(wq)
            if self.rational:
                self.Rqk.append(splines.basis_matrix(t, self.p, xq))
                self.Zk.append(splines.basis_matrix(t, self.p, g))
            else:
                wf = (lambda s, k=k: self.domain.weight1d(k, s))
                self.Rqk.append(nurbs_basis_1d(t, self.p, wf, xq))
                self.Zk.append(nurbs_basis_1d(t, self.p, wf, g))
        self.n = tuple(len(g) for g in self.gk)
        self.nqk = tuple(len(x) for x in self.xqk)
        self.N = int(np.prod(self.n))
        self.Nq = int(np.prod(self.nqk))
        g3, g2, g1 = np.meshgrid(self.gk[2], self.gk[1], self.gk[0], indexing="ij")
        self.ghat = np.stack([g1.ravel(), g2.ravel(), g3.ravel()], axis=-1)
        self.Xc = self.domain.map(self.ghat)
        q3, q2, q1 = np.meshgrid(self.xqk[2], self.xqk[1], self.xqk[0], indexing="ij")
        self.qhat = np.stack([q1.ravel(), q2.ravel(), q3.ravel()], axis=-1)
        self.Xq = self.domain.map(self.qhat)
        w3, w2, w1 = np.meshgrid(self.wqk[2], self.wqk[1], self.wqk[0], indexing="ij")
        self.W = (w1 * w2 * w3).ravel()
        self.J = np.abs(self.domain.detJ(self.qhat))
        if self.rational:
            self.Wq = self.domain.weight(self.qhat)       # B_j / W at the quadrature points
            self.Wg = self.domain.weight(self.ghat)       # and at the collocation points
            self._zfull = None
        else:
            self._zlu = [_LUSolve(Z) for Z in self.Zk]

    def gamma_matrix(self, rows=None):
        Xr = self.Xc if rows is None else self.Xc[rows]
        if callable(self.kernel):
            return self.kernel(Xr, self.Xq)
        return kernels.kernel_matrix(self.kernel, Xr, self.Xq, self.ell, self.sigma)

    def gamma_apply(self, Y, chunk=512):
        out = np.empty((self.N, Y.shape[1]))
        for s in range(0, self.N, chunk):
            rows = np.arange(s, min(s + chunk, self.N))
            out[rows] = self.gamma_matrix(rows) @ Y
        return out

    # -- dense (tiny meshes) ---------------------------------------------
    def Rq_dense(self):
        R = kron.kron3(*self.Rqk)
        return R / self.Wq[:, None] if self.rational else R

    def Z_dense(self):
        Z = kron.kron3(*self.Zk)
        return Z / self.Wg[:, None] if self.rational else Z

    def A_dense(self):
        return self.gamma_matrix() @ ((self.J * self.W)[:, None] * self.Rq_dense())

    def Aprime_dense(self):
        """Z^-1 A through a full LU with complete pivoting, P Z Q = L U."""
        Z = self.Z_dense()
        A = self.A_dense()
        P, L, U, Q = _complete_pivot_lu(Z)
        # A' = Q U^-1 L^-1 P A
        T = sla.solve_triangular(L, P @ A, lower=True, unit_diagonal=True)
        T = sla.solve_triangular(U, T, lower=False)
        return Q @ T

    # -- matrix-free Algorithm 1 ---------------------------------------------
    def apply_A(self, V, gamma_apply=None):
        V = np.asarray(V, dtype=np.float64)
        vec = V.ndim == 1
        if vec:
            V = V[:, None]
        y = kron.kron_apply(self.Rqk, V)                       # 1
        if self.rational:
            y = y / self.Wq[:, None]
        y = (self.J * self.W)[:, None] * y                      # 2
        z = (gamma_apply or self.gamma_apply)(y)                # 3
        return z[:, 0] if vec else z

    def solve_Z(self, X):
        X = np.asarray(X, dtype=np.float64)
        if self.rational:
            if self._zfull is None:
                self._zfull = _complete_pivot_lu(self.Z_dense())
            P, L, U, Q = self._zfull
            T = sla.solve_triangular(L, P @ X, lower=True, unit_diagonal=True)
            return Q @ sla.solve_triangular(U, T, lower=False)
        return kron.kron_solve(self._zlu, X)

    def apply_Aprime(self, V, gamma_apply=None):
        return self.solve_Z(self.apply_A(V, gamma_apply))       # 4

    def eig_dense(self, M=None):
        """Generalized non-symmetric eigenpairs (LAPACK dggev), sorted by
        descending real part."""
        lam, V = sla.eig(self.A_dense(), self.Z_dense())
        order = np.argsort(-lam.real, kind="stable")
        lam, V = lam[order], V[:, order]
        if M is not None:
            lam, V = lam[:M], V[:, :M]
        return lam, V


def _complete_pivot_lu(A):
    """P A Q = L U with complete pivoting (Gaussian elimination, textbook)."""
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    rp = np.arange(n)
    cp = np.arange(n)
    for k in range(n):
        sub = np.abs(A[k:, k:])
        i, j = np.unravel_index(np.argmax(sub), sub.shape)
        i += k
        j += k
        A[[k, i], :] = A[[i, k], :]
        rp[[k, i]] = rp[[i, k]]
        A[:, [k, j]] = A[:, [j, k]]
        cp[[k, j]] = cp[[j, k]]
        if A[k, k] != 0:
            A[k + 1:, k] /= A[k, k]
            A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    L = np.tril(A, -1) + np.eye(n)
    U = np.triu(A)
    P = np.eye(n)[rp]
    Q = np.eye(n)[:, cp]
    return P, L, U, Q
