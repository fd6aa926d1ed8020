"""Pins of the oracle's Galerkin-IBQ and collocation discretisations (no GPU).

Each pin is fixed by something other than the oracle itself: closed-form
spectra of finite-rank kernels, the analytic exponential-kernel spectrum,
exactness of interpolation based quadrature for kernels inside the
interpolation space, Kronecker structure, and structural invariants.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.integrate import quad

from oracle import analytic, collocation, errors, galerkin, geometry, kron, product1d
from oracle.kernels import EXPONENTIAL, GAUSSIAN

LO, HI = (0.0, -1.0, 0.5), (1.0, 1.0, 2.0)
CK = (1.0, 2.0, 3.0)


def _poly_kernel(X, Y):
    """Gamma = 1 + sum_k c_k x_k y_k: a rank-4 kernel with range span{1, x_k}."""
    return 1.0 + sum(CK[k] * np.outer(X[:, k], Y[:, k]) for k in range(3))


def _poly_kernel_spectrum():
    """Nonzero eigenvalues of the integral operator of _poly_kernel on the
    box [LO, HI]: eigenvalues of diag(c) G with G the Gram matrix of
    {1, x1, x2, x3} (closed-form monomial integrals)."""
    lo, hi = np.array(LO), np.array(HI)
    V = np.prod(hi - lo)
    mean = (lo + hi) / 2
    sq = (hi ** 3 - lo ** 3) / (3 * (hi - lo))
    G = np.zeros((4, 4))
    G[0, 0] = V
    G[0, 1:] = G[1:, 0] = V * mean
    for k in range(3):
        for m in range(3):
            G[1 + k, 1 + m] = V * (sq[k] if k == m else mean[k] * mean[m])
    C = np.diag([1.0, *CK])
    return np.sort(np.linalg.eigvals(C @ G).real)[::-1]


# ---------------------------------------------------------------- Kronecker
def test_kron_apply_and_solve_match_explicit_kronecker():
    rng = np.random.default_rng(0)
    mats = [rng.standard_normal((n, n)) + 3 * np.eye(n) for n in (3, 4, 5)]
    X = rng.standard_normal((60, 2))
    K = kron.kron3(*mats)
    assert np.abs(kron.kron_apply(mats, X) - K @ X).max() < 1e-12
    rect = [rng.standard_normal((m, n)) for m, n in ((2, 3), (5, 4), (3, 5))]
    assert np.abs(kron.kron_apply(rect, X) - kron.kron3(*rect) @ X).max() < 1e-12
    solvers = [galerkin._LUSolve(A) for A in mats]
    assert np.abs(kron.kron_solve(solvers, X) - np.linalg.solve(K, X)).max() < 1e-12


# ---------------------------------------------------------------- Galerkin
def test_galerkin_finite_rank_kernel_closed_form():
    dom = geometry.Box(LO, HI)
    ref = _poly_kernel_spectrum()
    for p in (1, 2):
        g = galerkin.GalerkinIBQ(dom, p, (2, 3, 2), _poly_kernel, None)
        lam, _ = g.eig_dense()
        assert np.abs(lam[:4] - ref).max() < 1e-11 * ref[0]
        assert np.abs(lam[4:]).max() < 1e-11 * ref[0]


def test_ibq_equals_gauss_galerkin_for_kernels_in_interpolation_space():
    dom = geometry.Box(LO, HI)

    def k2(X, Y):   # degree <= 2 per variable: inside S~ x S~ for p = 2
        return 1 + np.outer(X[:, 0], Y[:, 0]) + 2 * np.outer(X[:, 1] ** 2, Y[:, 1] ** 2) \
            + 3 * np.outer(X[:, 2], Y[:, 2])
    ibq = galerkin.GalerkinIBQ(dom, 2, (2, 2, 3), k2, None)
    gq = galerkin.GalerkinGauss(dom, 2, (2, 2, 3), k2, None)
    A1, A2 = ibq.A_dense(), gq.A_dense()
    assert np.abs(A1 - A2).max() < 1e-12 * np.abs(A2).max()
    # ... and for a Gaussian kernel it is only an approximation
    ibq = galerkin.GalerkinIBQ(dom, 2, (2, 2, 3), GAUSSIAN, 0.7)
    gq = galerkin.GalerkinGauss(dom, 2, (2, 2, 3), GAUSSIAN, 0.7, q1d=6)
    d = np.abs(ibq.A_dense() - gq.A_dense()).max() / np.abs(gq.A_dense()).max()
    assert 1e-9 < d < 1e-1


def test_gauss_galerkin_finite_rank_kernel_closed_form():
    # standard Galerkin with (p+1)-point Gauss rules is exact for this kernel
    dom = geometry.Box(LO, HI)
    ref = _poly_kernel_spectrum()
    for p in (1, 2, 3):
        g = galerkin.GalerkinGauss(dom, p, (2, 3, 2), _poly_kernel, None)
        lam, _ = g.eig_dense()
        assert np.abs(lam[:4] - ref).max() < 1e-11 * ref[0]
        assert np.abs(lam[4:]).max() < 1e-11 * ref[0]


@pytest.mark.parametrize("kind,ell", [(EXPONENTIAL, 1.0), (GAUSSIAN, 0.5)])
def test_gauss_galerkin_3d_dense_equals_product_of_1d(kind, ell):
    g = galerkin.GalerkinGauss(geometry.Box(LO, HI), 2, (3, 2, 2), kind, ell, sigma=1.2)
    lam, _ = g.eig_dense(15)
    ref = product1d.galerkin_gauss_box_spectrum(2, (3, 2, 2), kind, ell, sigma=1.2, M=15, lo=LO, hi=HI)
    assert np.abs(lam - ref).max() < 1e-12 * ref[0]
    # a different rule (4 points per element) changes the discretisation, consistently
    g4 = galerkin.GalerkinGauss(geometry.Box(LO, HI), 2, (3, 2, 2), kind, ell, sigma=1.2, q1d=4)
    ref4 = product1d.galerkin_gauss_box_spectrum(2, (3, 2, 2), kind, ell, sigma=1.2, M=15, lo=LO, hi=HI, nq=4)
    assert np.abs(g4.eig_dense(15)[0] - ref4).max() < 1e-12 * ref4[0]


def test_gauss_galerkin_standard_form_operator():
    # A' applied through the Kronecker Cholesky factors equals the assembled
    # L^-1 A L^-T with L the Cholesky factor of the assembled Z
    g = galerkin.GalerkinGauss(geometry.QuarterAnnulus(), 2, (2, 3, 2), GAUSSIAN, 0.6)
    L = np.linalg.cholesky(g.Z_dense())
    Ap = sla.solve_triangular(L, sla.solve_triangular(L, g.A_dense().T, lower=True).T, lower=True)
    X = np.random.default_rng(3).standard_normal((g.Bq.shape[1], 4))
    assert np.abs(g.apply_Aprime(X) - Ap @ X).max() < 1e-12 * np.abs(Ap @ X).max()
    # and its eigenvalues are those of the pencil (A, Z)
    lam = np.sort(np.linalg.eigvalsh(0.5 * (Ap + Ap.T)))[::-1][:8]
    assert np.abs(lam - g.eig_dense(8)[0]).max() < 1e-12 * lam[0]


def test_gauss_galerkin_constant_kernel_rank_one():
    g = galerkin.GalerkinGauss(geometry.Box(LO, HI), 2, (2, 3, 2), GAUSSIAN, np.inf, sigma=1.5)
    lam, _ = g.eig_dense()
    vol = np.prod(np.array(HI) - np.array(LO))
    assert abs(lam[0] - 2.25 * vol) < 1e-12 * lam[0]
    assert np.abs(lam[1:]).max() < 1e-12 * lam[0]


def test_constant_kernel_rank_one():
    # Gamma = sigma^2: lambda_1 = sigma^2 |D|, the rest vanish
    for dom, exact in ((geometry.Box(LO, HI), True), (geometry.QuarterAnnulus(), False)):
        g = galerkin.GalerkinIBQ(dom, 2, (2, 3, 2), GAUSSIAN, np.inf, sigma=1.5)
        lam, _ = g.eig_dense()
        if exact:
            assert abs(lam[0] - 2.25 * dom.volume()) < 1e-12 * lam[0]
            assert np.abs(lam[1:]).max() < 1e-12 * lam[0]
        else:   # sqrt J is only interpolated on the curved domain
            assert abs(lam[0] - 2.25 * dom.volume()) < 1e-3 * lam[0]


@pytest.mark.parametrize("kind,ell", [(EXPONENTIAL, 1.0), (GAUSSIAN, 0.5)])
def test_galerkin_3d_dense_equals_product_of_1d(kind, ell):
    g = galerkin.GalerkinIBQ(geometry.Box(LO, HI), 2, (3, 2, 2), kind, ell, sigma=1.2)
    lam, _ = g.eig_dense(15)
    ref = product1d.galerkin_box_spectrum(2, (3, 2, 2), kind, ell, sigma=1.2, M=15, lo=LO, hi=HI)
    assert np.abs(lam - ref).max() < 1e-12 * ref[0]


def test_nine_step_operator_equals_assembled_standard_form():
    g = galerkin.GalerkinIBQ(geometry.QuarterAnnulus(), 2, (2, 3, 2), EXPONENTIAL, 0.5)
    A, Z = g.A_dense(), g.Z_dense()
    L = np.linalg.cholesky(Z)
    Ap = np.linalg.solve(L, np.linalg.solve(L, A).T).T           # L^-1 A L^-T
    V = np.random.default_rng(1).standard_normal((g.N, 3))
    assert np.abs(g.apply_Aprime(V) - Ap @ V).max() < 1e-13 * np.abs(Ap).max()
    assert np.abs(g.apply_A(V) - A @ V).max() < 1e-13 * np.abs(A).max()


def test_galerkin_symmetric_psd_on_curved_domain():
    g = galerkin.GalerkinIBQ(geometry.QuarterAnnulus(), 3, (2, 2, 2), GAUSSIAN, 0.4)
    A = g.A_dense()
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > -1e-13 * np.abs(A).max()


def test_eigenvalues_linear_in_sigma2_and_scale_with_domain():
    lam1 = galerkin.GalerkinIBQ("cube", 2, (2, 2, 3), GAUSSIAN, 0.6, sigma=1.0).eig_dense(6)[0]
    lam2 = galerkin.GalerkinIBQ("cube", 2, (2, 2, 3), GAUSSIAN, 0.6, sigma=2.0).eig_dense(6)[0]
    assert np.abs(lam2 - 4 * lam1).max() < 1e-12 * lam2[0]
    s = 1.7   # scale domain and correlation length: lambda scales by s^3
    for dom, doms in ((geometry.QuarterAnnulus(1, 2, 1), geometry.QuarterAnnulus(s, 2 * s, s)),
                      (geometry.Box(LO, HI), geometry.Box(s * np.array(LO), s * np.array(HI)))):
        a = galerkin.GalerkinIBQ(dom, 2, (2, 2, 2), EXPONENTIAL, 0.5).eig_dense(6)[0]
        b = galerkin.GalerkinIBQ(doms, 2, (2, 2, 2), EXPONENTIAL, 0.5 * s).eig_dense(6)[0]
        assert np.abs(b - s ** 3 * a).max() < 1e-11 * b[0]


def test_galerkin_converges_to_analytic_exponential_spectrum():
    ref = analytic.exponential_1d(5, 1.0)[0]
    errs = []
    for nel in (8, 16, 32, 64):
        A, Z = product1d.galerkin_pencil_1d(2, nel, EXPONENTIAL, 1.0)
        lam = np.sort(sla.eigh(A, Z, eigvals_only=True))[::-1][:5]
        errs.append(errors.rel_errors(ref, lam))
    errs = np.array(errs)
    assert errs[-1].max() < 2e-3 and errs[-1][0] < 3e-5
    rate = errs[:-1, 0] / errs[1:, 0]
    assert np.all(rate > 3.5) and np.all(rate < 4.5)               # O(h^2)
    # 3D cube: eigenvalues are products, lambda_1 -> 0.403274 (l = 1)
    lam3 = product1d.galerkin_box_spectrum(2, (64, 64, 64), EXPONENTIAL, 1.0, M=4)
    assert np.abs(lam3 - analytic.exponential_box(4, 1.0)).max() / lam3[0] < 1e-4


def test_trace_tends_to_sigma2_volume():
    prev = None
    for nel in (5, 10, 20):
        tr = product1d.galerkin_box_trace(3, (nel,) * 3, GAUSSIAN, 0.5, sigma=1.3)
        err = abs(tr - 1.69)
        if prev is not None:
            assert err < prev
        prev = err
    assert prev < 2e-2
    g = galerkin.GalerkinIBQ("cube", 2, (3, 2, 2), GAUSSIAN, 0.5, sigma=1.3)
    tr3 = np.trace(np.linalg.solve(g.Z_dense(), g.A_dense()))
    assert abs(tr3 - product1d.galerkin_box_trace(2, (3, 2, 2), GAUSSIAN, 0.5, sigma=1.3)) < 1e-12


def test_analytic_eigenpairs_solve_the_integral_equation():
    lam, w, par = analytic.exponential_1d(6, 0.7)
    for i in range(6):
        phi = lambda y: analytic.exponential_1d_eigfun(w[i], par[i], y)
        for x in (0.1, 0.37, 0.8):
            lhs = quad(lambda y: np.exp(-abs(x - y) / 0.7) * phi(y), 0, x, epsabs=1e-13)[0] \
                + quad(lambda y: np.exp(-abs(x - y) / 0.7) * phi(y), x, 1, epsabs=1e-13)[0]
            assert abs(lhs - lam[i] * phi(x)) < 1e-10
        nrm = quad(lambda y: phi(y) ** 2, 0, 1)[0]
        assert abs(nrm - 1) < 1e-10


# -------------------------------------------------------------- collocation
def test_collocation_finite_rank_kernel_closed_form():
    ref = _poly_kernel_spectrum()
    c = collocation.Collocation(geometry.Box(LO, HI), 2, (2, 2, 3), _poly_kernel, None)
    lam, _ = c.eig_dense()
    assert np.abs(lam[:4] - ref).max() < 1e-11 * ref[0]
    assert np.abs(lam[4:]).max() < 1e-11 * ref[0]


def test_collocation_constant_kernel():
    c = collocation.Collocation(geometry.Box(LO, HI), 3, (2, 2, 2), GAUSSIAN, np.inf)
    lam, _ = c.eig_dense()
    assert abs(lam[0] - 3.0) < 1e-12 and np.abs(lam[1:]).max() < 1e-11
    an = geometry.QuarterAnnulus()
    c = collocation.Collocation(an, 3, (4, 2, 2), GAUSSIAN, np.inf)
    lam, _ = c.eig_dense()
    assert abs(lam[0] - an.volume()) < 1e-6 * an.volume()


def test_collocation_matrices_on_annulus():
    c = collocation.Collocation(geometry.QuarterAnnulus(), 3, (3, 2, 2), EXPONENTIAL, 0.5)
    Z = c.Z_dense()
    assert np.abs(Z.sum(axis=1) - 1).max() < 1e-14                  # NURBS partition of unity
    # Z from the 3D NURBS definition R_j = w_j B_j / sum_l w_l B_l at the points
    from oracle import splines
    ts = [splines.open_knots(3, e, 1) for e in c.nel]
    B = [splines.basis_matrix(t, 3, g) for t, g in zip(ts, c.gk)]
    w1 = np.linalg.solve(B[0], geometry.circle_weight(c.gk[0]))
    B3 = kron.kron3(*B)
    w3 = np.kron(np.ones(c.n[2] * c.n[1]), w1)
    Zdef = B3 * w3[None, :] / (B3 @ w3)[:, None]
    assert np.abs(Zdef - Z).max() < 1e-14
    # Algorithm 1 with per-mode LU equals the full complete-pivot LU form
    V = np.random.default_rng(2).standard_normal((c.N, 2))
    assert np.abs(c.apply_Aprime(V) - c.Aprime_dense() @ V).max() < 1e-12


@pytest.mark.parametrize("kind,ell", [(EXPONENTIAL, 1.0), (GAUSSIAN, 0.5)])
def test_collocation_3d_dense_equals_product_of_1d(kind, ell):
    c = collocation.Collocation(geometry.Box(LO, HI), 2, (2, 3, 2), kind, ell, sigma=0.8)
    lam, _ = c.eig_dense(12)
    ref = product1d.collocation_box_spectrum(2, (2, 3, 2), kind, ell, sigma=0.8, M=12, lo=LO, hi=HI)
    assert np.abs(lam - ref).max() < 1e-12 * abs(ref[0])


def test_collocation_converges_to_analytic_exponential_spectrum():
    ref = analytic.exponential_1d(5, 0.25)[0]
    errs = []
    for nel in (16, 32, 64):
        A, Z = product1d.collocation_pencil_1d(2, nel, EXPONENTIAL, 0.25)
        ev = sla.eig(A, Z, right=False)
        ev = ev[np.argsort(-ev.real)][:5]
        assert np.abs(ev.imag).max() == 0
        errs.append(errors.rel_errors(ref, ev))
    errs = np.array(errs)
    assert errs[-1].max() < 2e-3
    assert np.all(errs[:-1, 0] / errs[1:, 0] > 3.0)


def test_error_measures():
    ref = np.array([1.0, 0.5, 0.1, 1e-4])
    lam = np.array([1.0 + 1e-7, 0.5, 0.1 - 1e-8, 1e-4 + 1e-8])
    e = errors.rel_errors(ref, lam)
    assert np.allclose(e, [1e-7, 0, 1e-7, 1e-4])
    f = errors.floored_rel_errors(ref, lam, tau=1e-2)
    assert np.allclose(f, [1e-7, 0, 1e-7, 1e-6])
    assert errors.clusters([3, 2, 2 * (1 + 1e-10), 1]) == [[0], [1, 2], [3]]
