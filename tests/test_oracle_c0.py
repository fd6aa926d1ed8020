"""Pins of the FP64 oracle on geometries with C^0 lines (paper Sec. 4.1: the
interpolation space of the Galerkin method is C^-1 where the geometry is C^0;
the solution space is the same for both methods, C^0 there).

* Degrees of freedom: on the half cylinder (one C^0 line, the middle of the
  half circle) the rule reproduces the N and Ntilde that Tables 1 and 2 print
  (tests/golden/half_cylinder_dof_tables.json), nine of ten pairs exactly.
* One-sided B-spline rows at a C^-1 knot are the limits from each side, and
  both sides agree at a C^0 knot.
* A box parametrised with a kink (|det DF| jumps at xi = 1/2): for the
  constant kernel the IBQ matrix is exact only if the interpolation space is
  broken at the kink, so lambda_1 equals sigma^2 u^T Z^-1 u with
  u_j = int B_j sqrt|det DF| from per-element Gauss quadrature, and the
  standard Gauss Galerkin gives the same value; without the rule IBQ misses.
* The kinked box is the unit cube: with the exponential kernel its spectrum
  under the rule matches the plain cube's within the discretisation error
  (median 1e-3), and misses it by more than 1e-2 without the rule.
* The half cylinder's volume pi (r1^2 - r0^2) / 2 * length."""
import json
import pathlib

import numpy as np
import pytest

from oracle import collocation, galerkin, geometry, splines
from workloads import half_cylinder_net, kinked_box_net

GOLDEN = json.loads((pathlib.Path(__file__).parent / "golden" / "half_cylinder_dof_tables.json").read_text())


def _vol(net):
    return geometry.NurbsVolume(net["degree"], net["knots"], net["ctrl"])


def _sizes(dom, p, nel, kernel):
    """(N, Ntilde) of the Galerkin-IBQ spaces from the knot vectors alone."""
    lines = [geometry.c0_lines(dom, k) for k in range(3)]
    mult = galerkin.default_interp_mult(kernel, p)
    N = Nt = 1
    for k in range(3):
        t = splines.open_knots(p, nel[k], 1, lines=lines[k], line_mult=p)
        ti = splines.open_knots(p, nel[k], mult, lines=lines[k], line_mult=p + 1)
        N *= splines.num_basis(t, p)
        Nt *= splines.num_basis(ti, p)
    return N, Nt


def test_half_cylinder_lines_and_volume():
    hc = _vol(half_cylinder_net(8.0, 10.0, 15.0))
    assert hc.c0_lines(0) == (0.5,) and hc.c0_lines(1) == () and hc.c0_lines(2) == ()
    assert abs(hc.volume() - np.pi / 2 * (10.0 ** 2 - 8.0 ** 2) * 15.0) < 1e-9


@pytest.mark.parametrize("row", GOLDEN["table1"], ids=lambda r: f"t1c{r['case']}")
def test_table1_dof_counts(row):
    N, Nt = _sizes(_vol(half_cylinder_net()), row["p"], row["nel"], "exponential")
    assert N == row["N"]
    if row["ntilde_follows_rule"]:
        assert Nt == row["Ntilde"]


@pytest.mark.parametrize("row", GOLDEN["table2"], ids=lambda r: f"t2c{r['case']}")
def test_table2_dof_counts(row):
    assert _sizes(_vol(half_cylinder_net()), row["p"], row["nel"], "gaussian") == (row["N"], row["Ntilde"])


def test_discretisations_use_the_rule():
    dom = _vol(half_cylinder_net())
    g = galerkin.GalerkinIBQ(dom, 2, (4, 1, 1), "exponential", 5.0)
    assert (g.N, g.Nt) == ((2 + 4 + 1) * 3 * 3, (2 * 4 + 2) * 3 * 3)
    c = collocation.Collocation(dom, 2, (4, 1, 1), "exponential", 5.0)
    assert c.N == g.N
    gg = galerkin.GalerkinGauss(dom, 2, (4, 1, 1), "exponential", 5.0)
    assert gg.N == g.N


@pytest.mark.parametrize("p,c", [(1, 0.5), (2, 0.5), (3, 0.5), (3, 0.1), (4, 0.7)])
def test_one_sided_rows(p, c):
    t = splines.open_knots(p, 4, 1, lines=(c,), line_mult=p + 1)       # C^-1 at c
    x = np.array([c])
    L = splines.basis_matrix(t, p, x, left=[True])
    R = splines.basis_matrix(t, p, x)
    d = 1e-9
    assert np.abs(L - splines.basis_matrix(t, p, x - d)).max() < 1e-6
    assert np.abs(R - splines.basis_matrix(t, p, x + d)).max() < 1e-6
    assert abs(L.sum() - 1) < 1e-14 and abs(R.sum() - 1) < 1e-14
    assert np.abs(L - R).max() > 0.5                                    # the space is broken there
    gl = splines.greville_left(t, p)
    g = splines.greville(t, p)
    assert gl.sum() == 1 and g[gl][0] == c
    assert np.sum(g == c) == 2                                           # both sides sit on the line
    assert np.linalg.matrix_rank(splines.basis_matrix(t, p, g, left=gl)) == len(g)
    tc = splines.open_knots(p, 4, 1, lines=(c,), line_mult=p)            # C^0: the sides agree
    assert np.abs(splines.basis_matrix(tc, p, x, left=[True]) - splines.basis_matrix(tc, p, x)).max() < 1e-14
    assert not splines.greville_left(tc, p).any()


def _constant_kernel_reference(knots, p, kink, at):
    """sigma^2 = 1: u^T Z^-1 u with u_j = int B_j sqrt(x'(xi)) by per-element Gauss quadrature
    (exact: x' is constant on each side of the kink).  Directions 2 and 3 contribute 1."""
    xq, wq = splines.element_quadrature(np.union1d(knots, [kink]), p + 2)
    slope = np.where(xq < kink, at / kink, (1 - at) / (1 - kink))
    u = splines.basis_matrix(knots, p, xq).T @ (wq * np.sqrt(slope))
    Z = splines.mass_matrix(knots, p, knots, p)
    return u @ np.linalg.solve(Z, u)


@pytest.mark.parametrize("p,nel", [(2, (6, 2, 2)), (3, (4, 1, 2))])
def test_kinked_box_constant_kernel(p, nel):
    kink, at = 0.5, 0.3
    dom = _vol(kinked_box_net(kink, at))
    g = galerkin.GalerkinIBQ(dom, p, nel, "gaussian", np.inf)
    lam, _ = g.eig_dense()
    ref = _constant_kernel_reference(g.knots[0], p, kink, at)
    assert abs(lam[0] / ref - 1) < 1e-13
    assert np.abs(lam[1:]).max() < 1e-13 * lam[0]
    gg = galerkin.GalerkinGauss(dom, p, nel, "gaussian", np.inf)
    assert abs(gg.eig_dense(1)[0][0] / ref - 1) < 1e-13
    # interpolation space left continuous at the kink: the jump of sqrt|det DF| is not interpolated
    g0 = galerkin.GalerkinIBQ(dom, p, nel, "gaussian", np.inf, lines=[(), (), ()])
    ref0 = _constant_kernel_reference(g0.knots[0], p, kink, at)
    assert abs(g0.eig_dense(1)[0][0] / ref0 - 1) > 1e-4


def test_kinked_box_matches_cube():
    """Exponential kernel with the C^0 interpolation space of Sec. 4.1."""
    p, nel, ell = 2, (8, 3, 3), 0.5
    kinked = _vol(kinked_box_net(0.5, 0.3))
    lam_box = galerkin.GalerkinIBQ(geometry.Box(), p, nel, "exponential", ell).eig_dense(8)[0]
    lam = galerkin.GalerkinIBQ(kinked, p, nel, "exponential", ell).eig_dense(8)[0]
    lam0 = galerkin.GalerkinIBQ(kinked, p, nel, "exponential", ell, lines=[(), (), ()]).eig_dense(8)[0]
    assert np.median(np.abs(lam / lam_box - 1)) < 1e-3
    assert np.median(np.abs(lam0 / lam_box - 1)) > 1e-2
