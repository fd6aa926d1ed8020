"""Matrix-free isogeometric Galerkin method with interpolation based quadrature
(paper Sec. 3.1), plus the standard Gauss-quadrature Galerkin it replaces.

What is computed
----------------
Trial space (eq. trialspace): N_i = B_i(xh) / sqrt(|det DF(xh)|), tensor-product
B-splines B_i of degree p on the solution mesh.  Then the mass matrix is the
Kronecker product Z = Z_3 x Z_2 x Z_1 of univariate mass matrices and its
Cholesky factor is L = L_3 x L_2 x L_1.

Interpolation based quadrature (IBQ) factorises the covariance matrix as
    A = M^T B~^-1 J Gamma J B~^-T M,
with Gamma[a, c] = Gamma(F(g_a), F(g_c)) at the Greville points g of the
interpolation space S~ (degree p, continuity C^{p-1} for the Gaussian kernel
and C^0 for the exponential kernel), J = diag(sqrt|det DF(g_a)|),
B~ = B~_3 x B~_2 x B~_1 with (B~_k)[a, c] = B~_c(g_a) (rows are points), and
M = M_3 x M_2 x M_1 with (M_k)[a, j] = integral of B~_a B_j.

Where the geometry is only C^0 (a line xh_k = c, e.g. where two patches
meet), |det DF| jumps.  There the solution space is C^0 (knot multiplicity p)
and the interpolation space C^-1 (multiplicity p+1), Sec. 4.1; the two
interpolation points that then share the abscissa c are evaluated from their
own sides (basis rows and |det DF| as one-sided limits).

The standard-form operator (eq. standard with A' = L^-1 A L^-T, C = L^-T) is
applied in nine steps:
    L^-T, M, B~^-T, J, Gamma, J, B~^-1, M^T, L^-1.
The paper names the nine-step algorithm but does not print the order; the
order above is read off the factorisation.
"""
import numpy as np
import scipy.linalg as sla

from . import splines, kernels, kron
from .geometry import make_domain, c0_lines


class _TriSolve:
    """Solve with a triangular factor (optionally transposed) along one mode."""

    def __init__(self, L, lower, trans):
        self.L, self.lower, self.trans, self.n = L, lower, trans, L.shape[0]

    def __call__(self, X):
        return sla.solve_triangular(self.L, X, lower=self.lower, trans=self.trans)


class _LUSolve:
    def __init__(self, A, trans=0):
        self.lu = sla.lu_factor(A)
        self.trans, self.n = trans, A.shape[0]

    def __call__(self, X):
        return sla.lu_solve(self.lu, X, trans=self.trans)


def default_interp_mult(kernel, p):
    """C^0 interpolation space for the exponential kernel (Sec. 4.1), smooth
    C^{p-1} for the Gaussian kernel (Sec. 4.2)."""
    return p if kernel == kernels.EXPONENTIAL else 1


class GalerkinIBQ:
    """FP64 oracle of the Galerkin-IBQ discretisation on one tensor patch.

    Parameters
    ----------
    domain : geometry object (Box / QuarterAnnulus) or name
    p      : degree (same in all directions)
    nel    : 3-tuple of element counts
    kernel : "gaussian" | "exponential", or a callable Gamma(X, Y) -> matrix
    ell, sigma : kernel parameters
    interp_mult : interior knot multiplicity of the interpolation space
    lines  : per direction, the C^0 lines of the geometry (None: the domain's own)
    """

    def __init__(self, domain, p, nel, kernel, ell, sigma=1.0, interp_mult=None, lines=None):
        self.domain = make_domain(domain) if isinstance(domain, str) else domain
        self.p = int(p)
        self.nel = tuple(int(e) for e in nel)
        self.kernel, self.ell, self.sigma = kernel, ell, sigma
        if interp_mult is None:
            interp_mult = default_interp_mult(kernel, self.p) if isinstance(kernel, str) else 1
        self.interp_mult = interp_mult
        if lines is None:
            lines = [c0_lines(self.domain, k) for k in range(3)]
        self.lines = [tuple(l) for l in lines]
        self.knots, self.iknots = [], []
        self.Zk, self.Lk, self.Mk, self.Btk, self.gk, self.leftk = [], [], [], [], [], []
        for k, e in enumerate(self.nel):
            t = splines.open_knots(self.p, e, 1, lines=self.lines[k], line_mult=self.p)
            ti = splines.open_knots(self.p, e, interp_mult, lines=self.lines[k], line_mult=self.p + 1)
            g = splines.greville(ti, self.p)
            gl = splines.greville_left(ti, self.p)
            Zk = splines.mass_matrix(t, self.p, t, self.p)
            self.knots.append(t)
            self.iknots.append(ti)
            self.Zk.append(Zk)
            self.Lk.append(np.linalg.cholesky(Zk))
            self.Mk.append(splines.mass_matrix(ti, self.p, t, self.p))
            self.Btk.append(splines.basis_matrix(ti, self.p, g, left=gl))
            self.gk.append(g)
            self.leftk.append(gl)
        self.n = tuple(Z.shape[0] for Z in self.Zk)
        self.nt = tuple(len(g) for g in self.gk)
        self.N = int(np.prod(self.n))
        self.Nt = int(np.prod(self.nt))
        # interpolation points, flat index a = a1 + n1 (a2 + n2 a3)
        g3, g2, g1 = np.meshgrid(self.gk[2], self.gk[1], self.gk[0], indexing="ij")
        self.xhat = np.stack([g1.ravel(), g2.ravel(), g3.ravel()], axis=-1)
        l3, l2, l1 = np.meshgrid(self.leftk[2], self.leftk[1], self.leftk[0], indexing="ij")
        self.left = np.stack([l1.ravel(), l2.ravel(), l3.ravel()], axis=-1)
        self.X = self.domain.map(self.xhat, self.left)
        self.J = np.sqrt(np.abs(self.domain.detJ(self.xhat, self.left)))

    # -- kernel -----------------------------------------------------------
    def gamma_matrix(self, rows=None):
        Xr = self.X if rows is None else self.X[rows]
        if callable(self.kernel):
            return self.kernel(Xr, self.X)
        return kernels.kernel_matrix(self.kernel, Xr, self.X, self.ell, self.sigma)

    def gamma_apply(self, Y, chunk=2048):
        """Gamma @ Y, Gamma rows generated on the fly, chunk by chunk."""
        out = np.empty((self.Nt, Y.shape[1]))
        for s in range(0, self.Nt, chunk):
            rows = np.arange(s, min(s + chunk, self.Nt))
            out[rows] = self.gamma_matrix(rows) @ Y
        return out

    # -- dense assembly (tiny meshes) ------------------------------------
    def M_dense(self):
        return kron.kron3(*self.Mk)

    def Bt_dense(self):
        return kron.kron3(*self.Btk)

    def Z_dense(self):
        return kron.kron3(*self.Zk)

    def A_dense(self):
        """A = M^T B~^-1 J Gamma J B~^-T M, assembled densely."""
        M = self.M_dense()
        Bt = self.Bt_dense()
        G = self.J[:, None] * self.gamma_matrix() * self.J[None, :]
        BinvM = np.linalg.solve(Bt.T, M)           # B~^-T M
        return BinvM.T @ G @ BinvM

    # -- matrix-free nine-step operator ----------------------------------
    def _Lsolve(self, X, trans):
        return kron.kron_solve([_TriSolve(L, True, trans) for L in self.Lk], X)

    def _Btsolve(self, X, trans):
        return kron.kron_solve([_LUSolve(B, trans) for B in self.Btk], X)

    def apply_Aprime(self, Vp, gamma_apply=None):
        """A' V' = L^-1 M^T B~^-1 J Gamma J B~^-T M L^-T V' (nine steps)."""
        Vp = np.asarray(Vp, dtype=np.float64)
        vec = Vp.ndim == 1
        if vec:
            Vp = Vp[:, None]
        W = self._Lsolve(Vp, trans=1)              # 1  L^-T
        Y = kron.kron_apply(self.Mk, W)            # 2  M
        Y = self._Btsolve(Y, trans=1)              # 3  B~^-T
        Y = self.J[:, None] * Y                    # 4  J
        Z = (gamma_apply or self.gamma_apply)(Y)   # 5  Gamma
        Z = self.J[:, None] * Z                    # 6  J
        Z = self._Btsolve(Z, trans=0)              # 7  B~^-1
        U = kron.kron_apply([M.T for M in self.Mk], Z)  # 8  M^T
        out = self._Lsolve(U, trans=0)             # 9  L^-1
        return out[:, 0] if vec else out

    def apply_A(self, V, gamma_apply=None):
        """A V without the Cholesky transform."""
        V = np.asarray(V, dtype=np.float64)
        vec = V.ndim == 1
        if vec:
            V = V[:, None]
        Y = self._Btsolve(kron.kron_apply(self.Mk, V), trans=1)
        Z = self.J[:, None] * (gamma_apply or self.gamma_apply)(self.J[:, None] * Y)
        out = kron.kron_apply([M.T for M in self.Mk], self._Btsolve(Z, trans=0))
        return out[:, 0] if vec else out

    def solve_Z(self, X):
        return kron.kron_solve([_LUSolve(Z) for Z in self.Zk], X)

    def back_transform(self, Vp):
        """Eigenvector of the pencil from one of A': v = L^-T v'."""
        return self._Lsolve(np.asarray(Vp, dtype=np.float64), trans=1)

    def eig_dense(self, M=None):
        """Largest eigenpairs of the pencil (A, Z) by dense LAPACK (dsygvd)."""
        lam, V = sla.eigh(self.A_dense(), self.Z_dense())
        order = np.argsort(lam)[::-1]
        lam, V = lam[order], V[:, order]
        if M is not None:
            lam, V = lam[:M], V[:, :M]
        return lam, V


class GalerkinGauss:
    """Standard Galerkin with Gauss-Legendre quadrature (paper Sec. 3.1,
    eq. galerkin_system_matrices): the conventional method IBQ replaces.

    With the same trial space N_i = B_i / sqrt|det DF|:
      A_ij = sum_q sum_r w_q w_r B_i(q) sqrt J(q) Gamma(F q, F r) sqrt J(r) B_j(r)
    for tensor Gauss points q, r with `q1d` points per element and direction.
    """

    def __init__(self, domain, p, nel, kernel, ell, sigma=1.0, q1d=None):
        self.domain = make_domain(domain) if isinstance(domain, str) else domain
        self.p, self.nel = int(p), tuple(int(e) for e in nel)
        self.kernel, self.ell, self.sigma = kernel, ell, sigma
        q1d = q1d or (self.p + 1)
        Bq, xq, wq, Zk = [], [], [], []
        self.knots = []
        for k, e in enumerate(self.nel):
            # C^0 at the geometry's C^0 lines, as for IBQ
            t = splines.open_knots(self.p, e, 1, lines=c0_lines(self.domain, k), line_mult=self.p)
            self.knots.append(t)
            x, w = splines.element_quadrature(t, q1d)
            Bq.append(splines.basis_matrix(t, self.p, x))
            xq.append(x)
            wq.append(w)
            Zk.append(splines.mass_matrix(t, self.p, t, self.p))
        self.Bq = kron.kron3(*Bq)
        x3, x2, x1 = np.meshgrid(xq[2], xq[1], xq[0], indexing="ij")
        self.xhat = np.stack([x1.ravel(), x2.ravel(), x3.ravel()], axis=-1)
        self.X = self.domain.map(self.xhat)
        w3, w2, w1 = np.meshgrid(wq[2], wq[1], wq[0], indexing="ij")
        self.W = (w1 * w2 * w3).ravel()
        self.J = np.abs(self.domain.detJ(self.xhat))
        self.Zk = Zk
        self.N = self.Bq.shape[1]

    def A_dense(self):
        if callable(self.kernel):
            G = self.kernel(self.X, self.X)
        else:
            G = kernels.kernel_matrix(self.kernel, self.X, self.X, self.ell, self.sigma)
        s = self.W * np.sqrt(self.J)
        P = self.Bq * s[:, None]
        return P.T @ G @ P

    def Z_dense(self):
        return kron.kron3(*self.Zk)

    def apply_A(self, V):
        """A V with the assembled A (small meshes)."""
        return self.A_dense() @ V

    def apply_Aprime(self, Vp):
        """A' V' = L^-1 A L^-T V' with Z = L L^T, L = L_3 x L_2 x L_1 (Sec. 3.1)."""
        Lk = [np.linalg.cholesky(Z) for Z in self.Zk]
        W = kron.kron_solve([_TriSolve(L, True, 1) for L in Lk], Vp)
        return kron.kron_solve([_TriSolve(L, True, 0) for L in Lk], self.apply_A(W))

    def eig_dense(self, M=None):
        lam, V = sla.eigh(self.A_dense(), self.Z_dense())
        order = np.argsort(lam)[::-1]
        lam, V = lam[order], V[:, order]
        if M is not None:
            lam, V = lam[:M], V[:, :M]
        return lam, V
