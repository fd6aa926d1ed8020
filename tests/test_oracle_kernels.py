"""Pins of the oracle's covariance kernels and of its principal-angle helper (no GPU).

Kernels (Sec. 2 covariance function; Sec. 4.1 exponential, Sec. 4.2 Gaussian
kernel).  Both forms are fixed by closed-form integrals over the unit interval,
which a quadrature of the oracle's kernel matrix must reproduce:

  int_0^1 exp(-(x - y)^2 / l^2) dy = (l sqrt(pi) / 2) [erf(x / l) + erf((1 - x) / l)]
  int_0^1 exp(-|x - y| / l) dy     = l [2 - exp(-x / l) - exp(-(1 - x) / l)]

and over the unit cube by the product of three such factors (both kernels
factor over the coordinates).  A different length-scale convention, e.g.
exp(-d^2 / (2 l^2)), or a dropped sigma^2, fails these.  The C twin of the
kernel product (oracle/cmatvec.c) is pinned by the same integrals.

Principal angles (Sec. 4.1 compares eigenpairs; eigenvectors of degenerate
clusters are compared as subspaces): subspaces built with known principal
angles, in the Euclidean and in a G inner product.
"""
import numpy as np
import pytest
from scipy.special import erf

from oracle import cmatvec, errors, kernels, splines


def _composite_gauss(a, b, pieces, q, breaks=()):
    """Composite Gauss-Legendre rule on [a, b] with `pieces` equal panels,
    each further split at the given break points."""
    edges = np.unique(np.concatenate([np.linspace(a, b, pieces + 1),
                                      [x for x in breaks if a < x < b]]))
    xs, ws = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        x, w = splines.gauss_legendre(q, lo, hi)
        xs.append(x)
        ws.append(w)
    return np.concatenate(xs), np.concatenate(ws)


def _gauss_integral_1d(x, ell):
    return ell * np.sqrt(np.pi) / 2 * (erf(x / ell) + erf((1 - x) / ell))


def _exp_integral_1d(x, ell):
    return ell * (2 - np.exp(-x / ell) - np.exp(-(1 - x) / ell))


XS = np.array([0.0, 0.013, 0.25, 0.5, 0.731, 0.99, 1.0])


@pytest.mark.parametrize("ell", [0.1, 0.2, 0.5, 1.0, 2.0])
def test_gaussian_kernel_integral_1d(ell):
    y, w = _composite_gauss(0.0, 1.0, 64, 20)
    got = kernels.kernel_matrix(kernels.GAUSSIAN, XS, y, ell) @ w
    ref = _gauss_integral_1d(XS, ell)
    assert np.abs(got - ref).max() <= 1e-13 * ref.max()


@pytest.mark.parametrize("ell", [0.1, 0.25, 1.0, 2.0])
def test_exponential_kernel_integral_1d(ell):
    for x in XS:
        # the kernel has a kink at y = x: a panel edge there keeps the rule exact
        y, w = _composite_gauss(0.0, 1.0, 16, 20, breaks=(x,))
        got = kernels.kernel_matrix(kernels.EXPONENTIAL, [x], y, ell) @ w
        assert abs(got[0] - _exp_integral_1d(x, ell)) <= 1e-13


@pytest.mark.parametrize("kind", [kernels.GAUSSIAN, kernels.EXPONENTIAL])
@pytest.mark.parametrize("ell", [0.2, 0.5])
def test_kernel_integral_over_unit_cube(kind, ell):
    """3D points: the integral over the cube is the product of the 1D ones
    (sigma^2 in front); a tensor rule over product points of the cube."""
    rng = np.random.default_rng(3)
    X = rng.random((4, 3))
    sigma = 1.3
    got = []
    for x in X:
        # per direction, panel edges at the point's coordinate (kink of the L1 kernel)
        rules = [_composite_gauss(0.0, 1.0, 8, 12, breaks=(x[k],)) for k in range(3)]
        (y1, w1), (y2, w2), (y3, w3) = rules
        g3, g2, g1 = np.meshgrid(y3, y2, y1, indexing="ij")
        Y = np.stack([g1.ravel(), g2.ravel(), g3.ravel()], axis=-1)
        W = (w3[:, None, None] * w2[None, :, None] * w1[None, None, :]).ravel()
        got.append(float((kernels.kernel_matrix(kind, x[None, :], Y, ell, sigma) @ W)[0]))
    one = _gauss_integral_1d if kind == kernels.GAUSSIAN else _exp_integral_1d
    ref = sigma ** 2 * np.prod(one(X, ell), axis=1)
    assert np.abs(np.array(got) - ref).max() <= 1e-12 * ref.max()


@pytest.mark.parametrize("kind", [kernels.GAUSSIAN, kernels.EXPONENTIAL])
def test_c_kernel_product_integral(kind):
    """The C/OpenMP product with the quadrature weights as the block gives
    the same closed-form integrals (points on a line along each axis)."""
    ell, sigma = 0.3, 0.7
    y, w = _composite_gauss(0.0, 1.0, 64, 20, breaks=tuple(XS))
    one = _gauss_integral_1d if kind == kernels.GAUSSIAN else _exp_integral_1d
    for axis in range(3):
        Xr = np.full((len(XS), 3), 0.5)
        Xr[:, axis] = XS
        Xc = np.full((len(y), 3), 0.5)
        Xc[:, axis] = y
        Z = cmatvec.gamma_apply(kind, sigma, ell, Xr, Xc, np.stack([w, 2 * w], axis=1))
        ref = sigma ** 2 * one(XS, ell)
        assert np.abs(Z[:, 0] - ref).max() <= 1e-13
        assert np.abs(Z[:, 1] - 2 * ref).max() <= 2e-13


def test_gaussian_infinite_length_scale_is_constant():
    X = np.random.default_rng(1).random((5, 3))
    assert np.all(kernels.kernel_matrix(kernels.GAUSSIAN, X, X, np.inf, 1.5) == 2.25)


# ---------------------------------------------------------------- principal angles
def _rotated_pair(n, angles, rng):
    """Orthonormal U, V (n x k) with principal angles `angles`, in a random
    orthonormal frame: U = Q[:, :k], V_j = cos(a_j) U_j + sin(a_j) Q[:, k + j]."""
    k = len(angles)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    U = Q[:, :k]
    V = np.cos(angles)[None, :] * U + np.sin(angles)[None, :] * Q[:, k:2 * k]
    return U, V


def test_subspace_angle_is_the_largest_principal_angle():
    rng = np.random.default_rng(7)
    angles = np.array([0.05, 0.7, 0.3])
    U, V = _rotated_pair(9, angles, rng)
    # any bases of the two spans give the same angle
    Bu, Bv = rng.standard_normal((3, 3)), rng.standard_normal((3, 3))
    assert abs(errors.subspace_angle(U @ Bu, V @ Bv) - 0.7) < 1e-12
    assert abs(errors.subspace_angle(U, V) - 0.7) < 1e-12
    assert errors.subspace_angle(U, U @ Bu) < 1e-7
    # one vector each: the plain angle between them
    u, v = U[:, :1], V[:, 1:2]
    c = abs(float(u[:, 0] @ v[:, 0])) / np.linalg.norm(v)
    assert abs(errors.subspace_angle(u, v) - np.arccos(c)) < 1e-12


def test_subspace_angle_in_a_g_inner_product():
    """With G = L L^T, the G-angles between L^-T U0 and L^-T V0 are the
    Euclidean angles between U0 and V0."""
    rng = np.random.default_rng(8)
    n = 8
    A = rng.standard_normal((n, n))
    G = A @ A.T + n * np.eye(n)
    L = np.linalg.cholesky(G)
    U0, V0 = _rotated_pair(n, np.array([0.2, 0.45]), rng)
    U = np.linalg.solve(L.T, U0)
    V = np.linalg.solve(L.T, V0)
    assert abs(errors.subspace_angle(U, V, G) - 0.45) < 1e-12
    # the Euclidean angle of the mapped bases is a different number
    assert abs(errors.subspace_angle(U, V) - 0.45) > 1e-3
