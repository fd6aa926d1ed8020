"""Pins of the oracle's geometry maps (no GPU)."""
import numpy as np

from oracle import geometry, splines
from oracle.collocation import nurbs_basis_1d


def _quad3(n=16):
    x, w = splines.gauss_legendre(n, 0.0, 1.0)
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", w, w, w).ravel()
    return X, W


def test_annulus_lies_on_quarter_annulus():
    an = geometry.QuarterAnnulus(1.0, 2.0, 1.0)
    rng = np.random.default_rng(3)
    xh = rng.random((500, 3))
    x = an.map(xh)
    r = np.hypot(x[:, 0], x[:, 1])
    assert np.allclose(r, 1.0 + xh[:, 1], atol=1e-14)        # exact circle, r linear in eta
    th = np.arctan2(x[:, 1], x[:, 0])
    assert th.min() >= 0 and th.max() <= np.pi / 2
    assert np.allclose(x[:, 2], xh[:, 2])
    # end points of the quarter circle
    assert np.allclose(an.map(np.array([[0.0, 0, 0], [1.0, 0, 0]])), [[1, 0, 0], [0, 1, 0]], atol=1e-15)


def test_annulus_detJ_matches_finite_differences():
    an = geometry.QuarterAnnulus(1.0, 2.0, 1.3)
    rng = np.random.default_rng(4)
    xh = 0.05 + 0.9 * rng.random((50, 3))
    h = 1e-6
    for pt in xh:
        Jm = np.zeros((3, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jm[:, k] = (an.map(pt + e) - an.map(pt - e)) / (2 * h)
        assert abs(abs(np.linalg.det(Jm)) - an.detJ(pt)) < 1e-8 * an.detJ(pt)


def test_volumes():
    X, W = _quad3(20)
    an = geometry.QuarterAnnulus(1.0, 2.0, 1.0)
    assert abs(np.dot(an.detJ(X), W) - 3 * np.pi / 4) < 1e-12
    bx = geometry.Box((0, -1, 0.5), (1, 1, 2))
    assert abs(np.dot(bx.detJ(X), W) - 3.0) < 1e-13


def test_rational_weight_is_in_spline_space():
    # the NURBS denominator sum_l w_l B_l equals the circle's quadratic D(xi)
    for p in (2, 3, 4):
        t = splines.open_knots(p, 7, 1)
        g = splines.greville(t, p)
        w = np.linalg.solve(splines.basis_matrix(t, p, g), geometry.circle_weight(g))
        xs = np.linspace(0, 1, 41)
        assert np.abs(splines.basis_matrix(t, p, xs) @ w - geometry.circle_weight(xs)).max() < 1e-14
        R = nurbs_basis_1d(t, p, geometry.circle_weight, xs)
        assert np.abs(R.sum(axis=1) - 1).max() < 1e-14          # partition of unity
