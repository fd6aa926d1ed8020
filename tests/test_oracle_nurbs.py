"""Pins of the FP64 oracle on general single-patch NURBS volumes (paper
Sec. 3.2: NURBS geometry, and the full pivoted LU of Z when Z is not a
Kronecker product).

* The quarter annulus written as a NURBS control net reproduces the closed
  form (map, |det DF|, volume 3 pi / 4), and its spectra under both methods
  equal those of the closed-form domain (the rational trial space B_j / W
  spans the tensor-weight NURBS space there).
* |det DF| against central differences of the map; an affine control net is
  the identity.
* On a curved volume with non-tensor weights, the standard form through the
  complete-pivoting LU of the full Z (the paper's algorithm) equals the
  generalized eigenvalues of (A, Z) from LAPACK.
* The constant kernel gives rank one with lambda_1 = |D| as the quadrature
  is refined (the integrands are rational)."""
import numpy as np
import pytest

from oracle import collocation, galerkin, geometry
from workloads import nurbs_annulus_net, nurbs_blob_net


def _set_distance(a, b):
    """Largest distance from an element of a to its nearest element of b."""
    return np.abs(np.asarray(a)[:, None] - np.asarray(b)[None, :]).min(axis=1).max()


def _vol(net):
    return geometry.NurbsVolume(net["degree"], net["knots"], net["ctrl"])


def test_annulus_net_matches_closed_form():
    nv, an = _vol(nurbs_annulus_net(1.0, 2.0, 1.0)), geometry.QuarterAnnulus()
    xh = np.random.default_rng(0).random((300, 3))
    assert np.abs(nv.map(xh) - an.map(xh)).max() < 1e-14
    assert np.abs(nv.detJ(xh) - an.detJ(xh)).max() < 1e-13
    assert abs(nv.volume() - 3 * np.pi / 4) < 1e-13


def test_jacobian_against_finite_differences():
    nv = _vol(nurbs_blob_net(4, n=(5, 4, 4), degree=(3, 2, 2)))
    xh = 0.02 + 0.96 * np.random.default_rng(1).random((200, 3))
    h = 1e-6
    cols = []
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        cols.append((nv.map(xh + e) - nv.map(xh - e)) / (2 * h))
    fd = np.abs(np.linalg.det(np.stack(cols, axis=-1)))
    assert np.abs(fd - nv.detJ(xh)).max() < 1e-7 * fd.max()


def test_affine_net_is_identity():
    nv = _vol(nurbs_blob_net(0, n=(4, 5, 4), degree=(2, 3, 2), wiggle=0.0, wrange=(1.0, 1.0)))
    xh = np.random.default_rng(2).random((100, 3))
    assert np.abs(nv.map(xh) - xh).max() < 1e-14 and np.abs(nv.detJ(xh) - 1).max() < 1e-13
    assert np.abs(nv.weight(xh) - 1).max() < 1e-15


@pytest.mark.parametrize("kernel,ell", [("exponential", 0.5), ("gaussian", 0.7)])
def test_annulus_net_spectra_equal_closed_form(kernel, ell):
    nv, an = _vol(nurbs_annulus_net()), geometry.QuarterAnnulus()
    c1, c2 = collocation.Collocation(an, 2, (3, 2, 2), kernel, ell), collocation.Collocation(nv, 2, (3, 2, 2), kernel, ell)
    l1, _ = c1.eig_dense()
    l2, _ = c2.eig_dense()
    # as sets: a complex pair's order is not fixed by the sort on real parts
    assert _set_distance(l1[:30], l2[:40]) < 1e-12 * abs(l1[0])
    g1, g2 = galerkin.GalerkinIBQ(an, 2, (3, 2, 2), kernel, ell), galerkin.GalerkinIBQ(nv, 2, (3, 2, 2), kernel, ell)
    e1, _ = g1.eig_dense()
    e2, _ = g2.eig_dense()
    assert np.abs(e1[:30] - e2[:30]).max() < 1e-12 * e1[0]


@pytest.mark.parametrize("p,nel", [(2, (2, 2, 2)), (3, (2, 3, 2))])
def test_complete_pivot_lu_equals_generalized_eig(p, nel):
    c = collocation.Collocation(_vol(nurbs_blob_net(7)), p, nel, "gaussian", 0.6)
    Z = c.Z_dense()
    # the weights are not a tensor product: Z is not the Kronecker product of its factors
    Zk = np.kron(np.kron(c.Zk[2], c.Zk[1]), c.Zk[0])
    assert np.abs(Z - Zk).max() > 1e-2
    lam, _ = c.eig_dense()
    la = np.linalg.eigvals(c.Aprime_dense())
    la = la[np.argsort(-la.real, kind="stable")]
    assert _set_distance(lam[:20], la[:30]) < 1e-11 * abs(lam[0])
    # and the matrix-free operator with its complete-pivoting LU solve
    X = np.random.default_rng(3).standard_normal((c.N, 3))
    ref = np.linalg.solve(Z, c.A_dense() @ X)
    assert np.abs(c.apply_Aprime(X) - ref).max() < 1e-10 * np.abs(ref).max()


def test_constant_kernel_tends_to_volume():
    net = nurbs_blob_net(3)
    vol = _vol(net).volume()
    errs = []
    for nq in (3, 6):
        c = collocation.Collocation(_vol(net), 2, (2, 2, 2), "gaussian", np.inf, nq=nq)
        lam, _ = c.eig_dense()
        assert np.abs(lam[1:]).max() < 1e-12 * abs(lam[0])     # rank one
        errs.append(abs(lam[0] - vol) / vol)
    assert errs[0] < 1e-3 and errs[1] < 1e-2 * errs[0]
