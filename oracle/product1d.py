"""Exact spectra of separable kernels on boxes from univariate pencils.

On a box the map F is affine per coordinate and both workload kernels factor
across coordinates, Gamma(x, y) = sigma^2 prod_k g(x_k - y_k).  All matrices
of both methods are then Kronecker products (paper Sec. 3.1 for Z, B~, M;
Sec. 3.3 remark for collocation), so the generalized eigenvalues of the 3D
pencil are exactly sigma^2 * lambda1_i * lambda2_j * lambda3_k, products of
the eigenvalues of the three univariate pencils, and eigenvectors are
Kronecker products of univariate eigenvectors.
"""
import numpy as np
import scipy.linalg as sla

from . import splines, kernels
from .galerkin import default_interp_mult


def galerkin_pencil_1d(p, nel, kind, ell, interp_mult=None, a=0.0, b=1.0):
    """Univariate IBQ pencil (A_k, Z_k) on [a, b] (sigma = 1).

    A_k = M_k^T B~_k^-1 (j Gamma_k j) B~_k^-T M_k with j = sqrt(b - a)."""
    if interp_mult is None:
        interp_mult = default_interp_mult(kind, p)
    t = splines.open_knots(p, nel, 1)
    ti = splines.open_knots(p, nel, interp_mult)
    g = splines.greville(ti, p)
    Z = splines.mass_matrix(t, p, t, p)
    M = splines.mass_matrix(ti, p, t, p)
    Bt = splines.collocation_matrix(ti, p, g)
    x = a + (b - a) * g
    G = (b - a) * kernels.kernel_1d_factor(kind, x, x, ell)
    BinvM = np.linalg.solve(Bt.T, M)
    return BinvM.T @ G @ BinvM, Z


def galerkin_gauss_pencil_1d(p, nel, kind, ell, nq=None, a=0.0, b=1.0):
    """Univariate standard-Galerkin pencil with Gauss quadrature on both sides
    of the kernel (sigma = 1), trial space B_i / sqrt(b - a):
    A_k = B_q^T diag(w) (j Gamma_k j) diag(w) B_q with j = sqrt(b - a)."""
    nq = nq or p + 1
    t = splines.open_knots(p, nel, 1)
    xq, wq = splines.element_quadrature(t, nq)
    Bq = splines.basis_matrix(t, p, xq)
    Z = splines.mass_matrix(t, p, t, p)
    x = a + (b - a) * xq
    G = (b - a) * kernels.kernel_1d_factor(kind, x, x, ell)
    P = Bq * wq[:, None]
    return P.T @ G @ P, Z


def collocation_pencil_1d(p, nel, kind, ell, nq=None, a=0.0, b=1.0):
    """Univariate collocation pencil (A_k, Z_k) on [a, b] (sigma = 1)."""
    nq = nq or p + 1
    t = splines.open_knots(p, nel, 1)
    g = splines.greville(t, p)
    xq, wq = splines.element_quadrature(t, nq)
    Rq = splines.basis_matrix(t, p, xq)
    Z = splines.basis_matrix(t, p, g)
    G = kernels.kernel_1d_factor(kind, a + (b - a) * g, a + (b - a) * xq, ell)
    A = G @ (((b - a) * wq)[:, None] * Rq)
    return A, Z


def _top_products(lams, M):
    l1, l2, l3 = lams
    P = (l3[:, None, None] * l2[None, :, None] * l1[None, None, :]).ravel()
    order = np.argsort(-P, kind="stable")
    return P[order[:M]] if M is not None else P[order]


def galerkin_box_spectrum(p, nel, kind, ell, sigma=1.0, M=None, lo=(0, 0, 0), hi=(1, 1, 1),
                          interp_mult=None):
    lams = []
    for k in range(3):
        A, Z = galerkin_pencil_1d(p, nel[k], kind, ell, interp_mult, lo[k], hi[k])
        lams.append(np.sort(sla.eigh(A, Z, eigvals_only=True))[::-1])
    return sigma ** 2 * _top_products(lams, M)


def galerkin_gauss_box_spectrum(p, nel, kind, ell, sigma=1.0, M=None, lo=(0, 0, 0), hi=(1, 1, 1), nq=None):
    lams = []
    for k in range(3):
        A, Z = galerkin_gauss_pencil_1d(p, nel[k], kind, ell, nq, lo[k], hi[k])
        lams.append(np.sort(sla.eigh(A, Z, eigvals_only=True))[::-1])
    return sigma ** 2 * _top_products(lams, M)


def collocation_box_spectrum(p, nel, kind, ell, sigma=1.0, M=None, lo=(0, 0, 0), hi=(1, 1, 1),
                             nq=None):
    """Returns complex eigenvalue products sorted by descending real part.

    Univariate collocation spectra are real for these kernels in practice;
    the imaginary parts are returned so that callers can check that."""
    lams = []
    for k in range(3):
        A, Z = collocation_pencil_1d(p, nel[k], kind, ell, nq, lo[k], hi[k])
        ev = sla.eig(A, Z, right=False)
        lams.append(ev[np.argsort(-ev.real, kind="stable")])
    l1, l2, l3 = lams
    P = (l3[:, None, None] * l2[None, :, None] * l1[None, None, :]).ravel()
    order = np.argsort(-P.real, kind="stable")
    P = sigma ** 2 * P[order]
    return P[:M] if M is not None else P


def galerkin_box_trace(p, nel, kind, ell, sigma=1.0, lo=(0, 0, 0), hi=(1, 1, 1), interp_mult=None):
    """Sum of all generalized eigenvalues = sigma^2 prod_k tr(Z_k^-1 A_k)."""
    tr = sigma ** 2
    for k in range(3):
        A, Z = galerkin_pencil_1d(p, nel[k], kind, ell, interp_mult, lo[k], hi[k])
        tr *= np.trace(np.linalg.solve(Z, A))
    return tr
