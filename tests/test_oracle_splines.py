"""Pins of the oracle's univariate spline machinery against library routines,
closed forms and identities (no GPU)."""
import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import splines


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
@pytest.mark.parametrize("mult", ["smooth", "c0"])
def test_basis_matches_scipy(p, mult):
    m = 1 if mult == "smooth" else p
    t = splines.open_knots(p, 7, m)
    x = np.concatenate([np.linspace(0, 1, 57), [0.0, 1.0, 3 / 7, 0.999999]])
    ours = splines.basis_matrix(t, p, x)
    ref = BSpline.design_matrix(x, t, p).toarray()
    assert np.abs(ours - ref).max() < 1e-13


@pytest.mark.parametrize("p,nel,mult,n", [(2, 8, 1, 10), (3, 20, 1, 23), (2, 8, 2, 17), (3, 20, 3, 61),
                                          (4, 32, 4, 129), (4, 16, 4, 65)])
def test_dimension_counts(p, nel, mult, n):
    assert splines.num_basis(splines.open_knots(p, nel, mult), p) == n


@pytest.mark.parametrize("p", [2, 3, 4])
@pytest.mark.parametrize("m", [1, 2])
def test_partition_of_unity_and_greville_reproduction(p, m):
    t = splines.open_knots(p, 9, min(m, p))
    x = np.linspace(0, 1, 101)
    B = splines.basis_matrix(t, p, x)
    g = splines.greville(t, p)
    assert np.abs(B.sum(axis=1) - 1).max() < 1e-14
    assert np.abs(B @ g - x).max() < 1e-14          # sum_i g_i B_i(x) = x


@pytest.mark.parametrize("q", [1, 2, 3, 5, 8])
def test_gauss_legendre_exact_for_polynomials(q):
    x, w = splines.gauss_legendre(q, 0.25, 1.75)
    for k in range(2 * q):
        exact = (1.75 ** (k + 1) - 0.25 ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13 * max(1, exact)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_mass_matrices_integrate_monomials(p):
    t = splines.open_knots(p, 6, 1)
    ti = splines.open_knots(p, 6, p)
    Z = splines.mass_matrix(t, p, t, p)
    M = splines.mass_matrix(ti, p, t, p)
    g, gi = splines.greville(t, p), splines.greville(ti, p)
    one, onei = np.ones(len(g)), np.ones(len(gi))
    assert abs(one @ Z @ one - 1.0) < 1e-14          # integral of 1
    assert abs(g @ Z @ g - 1.0 / 3.0) < 1e-14        # integral of x * x
    assert abs(onei @ M @ one - 1.0) < 1e-14
    assert abs(gi @ M @ g - 1.0 / 3.0) < 1e-14
    assert abs(onei @ M @ g - 0.5) < 1e-14           # integral of 1 * x
    assert np.allclose(Z, Z.T, atol=1e-16)
    assert np.linalg.eigvalsh(Z).min() > 0


@pytest.mark.parametrize("p", [2, 3, 4])
def test_collocation_matrix_identities(p):
    ti = splines.open_knots(p, 5, 1)
    g = splines.greville(ti, p)
    Bt = splines.collocation_matrix(ti, p, g)
    assert np.abs(Bt.sum(axis=1) - 1).max() < 1e-14
    assert np.abs(Bt @ g - g).max() < 1e-14          # interpolates x exactly
    # interpolation of a degree-p polynomial is exact
    f = lambda s: 1 + s - 2 * s ** 2 + 0.5 * s ** p
    c = np.linalg.solve(Bt, f(g))
    xs = np.linspace(0, 1, 33)
    assert np.abs(splines.basis_matrix(ti, p, xs) @ c - f(xs)).max() < 1e-12


def test_element_quadrature_ordering():
    t = splines.open_knots(2, 3, 1)
    x, w = splines.element_quadrature(t, 3)
    assert len(x) == 9 and np.all(np.diff(x) > 0)
    assert abs(w.sum() - 1) < 1e-15
    assert np.all((x[:3] < 1 / 3) & (x[3:6] > 1 / 3) & (x[3:6] < 2 / 3) & (x[6:] > 2 / 3))
