"""Pins of the extruded-domain product oracle (oracle/extruded.py), no GPU.

The cross-section x extrusion factorisation is checked against things other
than itself: the 3D dense oracles (GalerkinIBQ / Collocation assembled on the
whole quarter annulus, themselves pinned in test_oracle_methods.py and
test_oracle_geometry.py), the product-of-1D oracle on a box, and the ARPACK
reference of the full-size annulus (matrix-free nine-step operator with the C
kernel product, tests/golden/make_annulus_reference.py).
"""
import json
import os

import numpy as np
import pytest

from oracle import collocation, extruded, galerkin, geometry, product1d

HERE = os.path.dirname(os.path.abspath(__file__))


def _as_multiset(z):
    z = np.asarray(z, dtype=complex)
    return z[np.lexsort((np.round(z.imag, 11), np.round(z.real, 11)))]


@pytest.mark.parametrize("kind,ell", [("gaussian", 0.5), ("exponential", 0.4)])
@pytest.mark.parametrize("p,nel", [(2, (4, 3, 2)), (3, (3, 3, 2))])
def test_annulus_matches_3d_dense(kind, ell, p, nel):
    ann = geometry.QuarterAnnulus(1.0, 2.0, 1.3)
    lam_g, _ = galerkin.GalerkinIBQ(ann, p, nel, kind, ell, sigma=1.2).eig_dense()
    got_g = extruded.galerkin_spectrum(ann, p, nel, kind, ell, sigma=1.2)
    assert len(got_g) == len(lam_g)
    assert np.abs(np.sort(lam_g)[::-1] - got_g).max() <= 1e-12 * abs(lam_g).max()
    lam_c, _ = collocation.Collocation(ann, p, nel, kind, ell, sigma=1.2).eig_dense()
    got_c = extruded.collocation_spectrum(ann, p, nel, kind, ell, sigma=1.2)
    assert len(got_c) == len(lam_c)
    assert np.abs(_as_multiset(lam_c) - _as_multiset(got_c)).max() <= 1e-12 * abs(lam_c).max()


@pytest.mark.parametrize("kind,ell", [("gaussian", 0.3), ("exponential", 0.7)])
def test_box_matches_product_of_1d(kind, ell):
    lo, hi = (0.0, -1.0, 0.5), (1.0, 1.0, 2.0)
    box = geometry.Box(lo, hi)
    nel = (5, 4, 3)
    ref = product1d.galerkin_box_spectrum(2, nel, kind, ell, sigma=0.9, lo=lo, hi=hi)
    got = extruded.galerkin_spectrum(box, 2, nel, kind, ell, sigma=0.9)
    assert np.abs(ref - got).max() <= 1e-12 * ref[0]
    refc = product1d.collocation_box_spectrum(3, nel, kind, ell, sigma=0.9, lo=lo, hi=hi)
    gotc = extruded.collocation_spectrum(box, 3, nel, kind, ell, sigma=0.9)
    assert np.abs(_as_multiset(refc) - _as_multiset(gotc)).max() <= 1e-12 * abs(refc[0])


def test_other_domains_are_refused():
    with pytest.raises(ValueError):
        extruded.extrusion(object())


def test_full_size_annulus_matches_arpack_reference():
    """p = 4, 32 x 32 x 16 (N = 25920), Gaussian ell = 0.5: the product oracle
    against ARPACK on the matrix-free operator (a different route)."""
    with open(os.path.join(HERE, "golden", "annulus_p4_32x32x16_gaussian_l0.5_galerkin.json")) as f:
        ref = np.array(json.load(f)["lambda"])
    got = extruded.galerkin_spectrum(geometry.QuarterAnnulus(1.0, 2.0, 1.0), 4, (32, 32, 16), "gaussian", 0.5,
                                     M=len(ref))
    assert np.abs((got - ref) / ref).max() <= 1e-11


def test_stored_annulus_spectra_match_the_product_oracle():
    """The stored full-size spectra (tests/golden/make_annulus_spectra.py)
    are what the product oracle gives (the two cheaper problems recomputed)."""
    with open(os.path.join(HERE, "golden", "annulus_p4_32x32x16_spectra.json")) as f:
        rec = json.load(f)
    ann = geometry.QuarterAnnulus(1.0, 2.0, 1.0)
    g = rec["spectra"]["galerkin-gaussian"]
    got = extruded.galerkin_spectrum(ann, 4, (32, 32, 16), "gaussian", g["ell"], M=len(g["lambda"]))
    assert np.abs(got - np.array(g["lambda"])).max() <= 1e-14 * got[0]
    c = rec["spectra"]["collocation-exponential"]
    gotc = extruded.collocation_spectrum(ann, 4, (32, 32, 16), "exponential", c["ell"], M=len(c["lambda"]))
    assert np.abs(gotc.real - np.array(c["lambda"])).max() <= 1e-14 * abs(gotc[0])
    assert np.abs(gotc.imag).max() <= 1e-12 * abs(gotc[0])
