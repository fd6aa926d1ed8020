"""Pins of the oracle's truncated K-L expansion (paper Sec. 2, eq. kle).

* Galerkin eigenvectors from the dense generalized solve are Z-orthonormal,
  so their eigenfunctions (B-splines over sqrt|det DF|) have unit L^2(D) norm:
  checked on the curved annulus, where the 1/sqrt J scaling matters.
* The pointwise variance of the truncated field integrates to sum lambda_i
  (orthonormal eigenfunctions), with a finer, independent Gauss rule.
* The leading eigenfunction on the unit cube with the L1-exponential kernel
  converges to the product of Ghanem & Spanos' closed-form 1D modes.
* Unit draws return sqrt(lambda_i) phi_i; many seeded N(0,1) draws reproduce
  the mean and the covariance sum_i lambda_i phi_i(x) phi_i(y) statistically."""
import numpy as np
import pytest

from oracle import analytic, collocation, galerkin, geometry, kl, splines
from workloads import nurbs_blob_net


def _fine_integral(disc, f_at, q):
    rules = [splines.element_quadrature(splines.open_knots(disc.p, e, 1), q) for e in disc.nel]
    grid = [r[0] for r in rules]
    w3, w2, w1 = np.meshgrid(rules[2][1], rules[1][1], rules[0][1], indexing="ij")
    w = (w1 * w2 * w3).ravel() * np.abs(disc.domain.detJ(kl.grid_points(grid)))
    return np.tensordot(w, f_at(grid), axes=1)


@pytest.mark.parametrize("cls", [galerkin.GalerkinIBQ, galerkin.GalerkinGauss])
def test_galerkin_eigenfunctions_are_orthonormal(cls):
    d = cls(geometry.QuarterAnnulus(), 2, (3, 2, 2), "exponential", 0.5)
    lam, V = d.eig_dense(12)
    assert np.abs(kl.l2_norms(d, V) - 1).max() < 1e-12
    # and mutually orthogonal in L^2(D): Gram matrix by the finer rule
    G = _fine_integral(d, lambda g: kl.eigenfunctions(d, V, g)[:, :, None] * kl.eigenfunctions(d, V, g)[:, None, :],
                       d.p + 4)
    assert np.abs(G - np.eye(12)).max() < 1e-11


@pytest.mark.parametrize("make", [
    lambda: galerkin.GalerkinIBQ(geometry.QuarterAnnulus(), 2, (3, 2, 2), "exponential", 0.5),
    lambda: collocation.Collocation(geometry.Box(), 3, (2, 3, 2), "gaussian", 0.7),
])
def test_integrated_variance_is_sum_of_eigenvalues(make):
    d = make()
    lam, V = d.eig_dense(10)
    lam, V = lam.real, V.real
    nrm = kl.l2_norms(d, V)
    var = lambda g: (kl.eigenfunctions(d, V, g) / nrm) ** 2 @ lam
    assert abs(_fine_integral(d, var, d.p + 5) - lam.sum()) < 1e-12 * lam.sum()


def test_leading_eigenfunction_converges_to_closed_form():
    lam1, w1, par1 = analytic.exponential_1d(1, 1.0)
    grid = [np.linspace(0, 1, 9)] * 3
    xh = kl.grid_points(grid)
    ref = np.prod([analytic.exponential_1d_eigfun(w1[0], par1[0], xh[:, k]) for k in range(3)], axis=0)
    for cls, bar in ((galerkin.GalerkinIBQ, 1e-3), (collocation.Collocation, 2e-3)):
        errs = []
        for nel in (4, 8):
            d = cls(geometry.Box(), 2, (nel,) * 3, "exponential", 1.0)
            lam, V = d.eig_dense(1)
            phi = kl.eigenfunctions(d, V.real, grid)[:, 0] / kl.l2_norms(d, V.real)[0]
            errs.append(np.abs(phi * np.sign(phi @ ref) - ref).max())
        assert errs[1] < bar and errs[1] < errs[0] / 2.5, errs


def test_unit_draws_and_statistics():
    d = collocation.Collocation(geometry.NurbsVolume(**{k: nurbs_blob_net(2)[k] for k in ("degree", "knots", "ctrl")}),
                                2, (2, 2, 2), "gaussian", 0.6)
    lam, V = d.eig_dense(6)
    lam, V = lam.real, V.real
    grid = [np.array([0.1, 0.5, 0.9])] * 3
    phi = kl.eigenfunctions(d, V, grid) / kl.l2_norms(d, V)
    F = kl.sample(d, lam, V, grid, np.eye(6), mu=2.0)
    assert np.abs(F - (2.0 + phi * np.sqrt(lam))).max() < 1e-13
    S = 40000
    xi = np.random.default_rng(7).standard_normal((6, S))
    F = kl.sample(d, lam, V, grid, xi, mu=0.5)
    C = (phi * lam) @ phi.T
    sd = np.sqrt(np.diag(C))
    assert np.abs(F.mean(axis=1) - 0.5).max() < 5 * sd.max() / np.sqrt(S)
    Ce = np.cov(F)
    assert np.abs(Ce - C).max() < 6 * C.max() * np.sqrt(2.0 / S)
