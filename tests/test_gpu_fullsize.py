"""Parity at the workloads' full sizes, in the launch configurations the
benchmark times: the fused kernel product on sampled output rows (each row
computed by the FP64 oracle over all columns), and complete K-L solves
against exact spectra: products of univariate pencils on the cube, of
cross-section and extrusion pencils on the quarter annulus (oracle/extruded.py),
and ARPACK on the annulus with the Gaussian kernel.

Kernel-product bar as in test_gpu_gamma (|err| <= tol * |Gamma| |Y|): FP32
chains of at most 32 MFMAs (128 columns) feed FP64 running totals, so the
FP32 bar does not grow with the column count: 1e-5.
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_2101_00629_amd as K
from oracle import cmatvec, collocation, errors, galerkin, geometry, product1d
from workloads import annulus_p4, cube_p2_64, cube_p3_20, normal_block

pytestmark = pytest.mark.gpu

TOL = {K.KA_FP32: 1e-5, K.KA_BF16X3: 6e-5}


def _points(p):
    if p["method"] == "galerkin":
        o = galerkin.GalerkinIBQ("cube", p["p"], p["nel"], p["kernel"], p["ell"])
        return o.X, o.X
    o = collocation.Collocation("cube", p["p"], p["nel"], p["kernel"], p["ell"])
    return o.Xc, o.Xq


def _sampled_check(p, precision, nsample=48, seed=0):
    Xr, Xc = _points(p)
    _sampled_rows(p, Xr, Xc, precision, nsample, seed)


def _sampled_rows(p, Xr, Xc, precision, nsample=48, seed=0):
    b = p["block"]
    Y = normal_block(seed + 1, len(Xc), b, dtype=np.float32)
    kid = K.KERNELS[p["kernel"]]
    xr = torch.tensor(Xr, dtype=torch.float32, device="cuda")
    xc = torch.tensor(Xc, dtype=torch.float32, device="cuda")
    y = torch.tensor(Y, device="cuda")
    z = torch.empty((len(Xr), b), dtype=torch.float32, device="cuda")
    nbytes = K.ka_gamma_workspace(len(Xr), len(Xc), b, precision)
    work = torch.empty(max(nbytes // 4, 1), dtype=torch.float32, device="cuda")
    K.ka_gamma_apply(kid, 1.0, p["ell"], xr, xc, y, z, precision, work)
    torch.cuda.synchronize()
    rows = np.random.default_rng(seed).choice(len(Xr), nsample, replace=False)
    rows[0], rows[-1] = 0, len(Xr) - 1
    Z = z.cpu().numpy()[rows].astype(np.float64)
    Xr32 = Xr[rows].astype(np.float32).astype(np.float64)
    Xc32 = Xc.astype(np.float32).astype(np.float64)
    ref = cmatvec.gamma_apply(p["kernel"], 1.0, p["ell"], Xr32, Xc32, Y.astype(np.float64))
    scale = cmatvec.gamma_apply(p["kernel"], 1.0, p["ell"], Xr32, Xc32, np.abs(Y.astype(np.float64)))
    err = (np.abs(Z - ref) / scale).max()
    print(p["name"], precision, "max scaled err", err)
    assert np.isfinite(Z).all() and err < TOL[precision]


@pytest.mark.parametrize("precision", [K.KA_FP32, K.KA_BF16X3])
def test_gamma_cube_p3_20_galerkin_exponential_c0(precision):
    _sampled_check(cube_p3_20("galerkin", "exponential"), precision)     # 226981 x 226981


@pytest.mark.parametrize("precision", [K.KA_FP32, K.KA_BF16X3])
def test_gamma_cube_p3_20_collocation_gaussian(precision):
    _sampled_check(cube_p3_20("collocation", "gaussian"), precision)     # 12167 x 512000


@pytest.mark.parametrize("precision", [K.KA_FP32, K.KA_BF16X3])
def test_gamma_cube_p2_64_galerkin_gaussian(precision):
    _sampled_check(cube_p2_64("galerkin"), precision, nsample=24)        # 287496 x 287496, b = 64


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-6), ("bf16x3", 1e-5)])
@pytest.mark.parametrize("method,kernel", [("galerkin", "gaussian"), ("galerkin", "exponential"),
                                           ("collocation", "gaussian"), ("collocation", "exponential")])
def test_cube_p3_20_solves(method, kernel, precision, bar):
    p = cube_p3_20(method, kernel, precision=precision)
    prob = K.Problem(K.desc_from_problem(p, seed=1000))
    rc, lam, info = K.ka_eigs(prob.h, p["M"], tol=1e-5, maxit=60)
    prob.close()
    if method == "galerkin":
        ref = product1d.galerkin_box_spectrum(p["p"], p["nel"], kernel, p["ell"], M=p["M"])
        lr = lam
    else:
        ref = product1d.collocation_box_spectrum(p["p"], p["nel"], kernel, p["ell"], M=p["M"]).real
        lr = lam[0::2]
        assert np.abs(lam[1::2]).max() <= 1e-6 * lr[0]
    err = errors.floored_rel_errors(ref, lr)
    print(p["name"], precision, info, "floored", err.max(), "raw", errors.rel_errors(ref, lr).max())
    assert rc == 0 and err.max() < bar


# ---- curved domain: quarter annulus, p = 4, 32 x 32 x 16, M = 100, b = 32 ----------------
GOLDEN_ANNULUS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                              "annulus_p4_32x32x16_gaussian_l0.5_galerkin.json")


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-6), ("bf16x3", 1e-5)])
def test_annulus_p4_galerkin_gaussian_solve(precision, bar):
    """Full-size solve against the stored FP64 oracle spectrum (ARPACK on the
    oracle's nine-step operator, written by tests/golden/make_annulus_reference.py)."""
    with open(GOLDEN_ANNULUS) as f:
        ref = np.array(json.load(f)["lambda"])
    p = annulus_p4("galerkin", "gaussian", precision=precision)
    prob = K.Problem(K.desc_from_problem(p, seed=2024))
    assert prob.N == 25920
    rc, lam, info = K.ka_eigs(prob.h, p["M"], tol=1e-5, maxit=80)
    prob.close()
    err = errors.floored_rel_errors(ref, lam)
    print(p["name"], precision, info, "floored", err.max(), "raw", errors.rel_errors(ref, lam).max())
    assert rc == 0 and err.max() < bar


def _annulus_points(p):
    dom = geometry.QuarterAnnulus()
    if p["method"] == "galerkin":
        o = galerkin.GalerkinIBQ(dom, p["p"], p["nel"], p["kernel"], p["ell"])
        return o.X, o.X
    o = collocation.Collocation(dom, p["p"], p["nel"], p["kernel"], p["ell"])
    return o.Xc, o.Xq


@pytest.mark.parametrize("method", ["galerkin", "collocation"])
def test_gamma_annulus_p4_exponential_sampled(method):
    """Kernel product at the full annulus sizes (Galerkin: 1,081,665 C0 points;
    collocation: 25,920 x 2,048,000) on sampled rows."""
    p = annulus_p4(method, "exponential")
    Xr, Xc = _annulus_points(p)
    _sampled_rows(p, Xr, Xc, K.KA_FP32, nsample=8 if method == "galerkin" else 32)


GOLDEN_ANNULUS_ALL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                  "annulus_p4_32x32x16_spectra.json")


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-6), ("bf16x3", 1e-5)])
@pytest.mark.parametrize("method,kernel", [("collocation", "gaussian"), ("collocation", "exponential"),
                                           ("galerkin", "exponential")])
def test_annulus_p4_solves_against_product_oracle(method, kernel, precision, bar):
    """Full-size annulus solves (collocation: 25,920 x 2,048,000 kernel pairs
    per block product; Galerkin exponential: 1,081,665^2) against the exact
    FP64 spectra of the oracle's cross-section x extrusion factorisation
    (tests/golden/make_annulus_spectra.py)."""
    with open(GOLDEN_ANNULUS_ALL) as f:
        ref = np.array(json.load(f)["spectra"][f"{method}-{kernel}"]["lambda"])
    p = annulus_p4(method, kernel, precision=precision)
    prob = K.Problem(K.desc_from_problem(p, seed=77))
    rc, lam, info = K.ka_eigs(prob.h, p["M"], tol=1e-5, maxit=80)
    prob.close()
    if method == "collocation":
        assert np.abs(lam[1::2]).max() <= 1e-6 * lam[0]
        lam = lam[0::2]
    err = errors.floored_rel_errors(ref[:p["M"]], lam)
    print(p["name"], precision, info, "floored", err.max(), "raw", errors.rel_errors(ref[:p["M"]], lam).max())
    assert rc == 0 and err.max() < bar


# ---- large matrix-free case: cube p = 2, 64^3 (N = 287,496), Gaussian l = 0.2, M = 200, b = 64 ----
@pytest.mark.parametrize("precision,bar", [("fp32", 1e-6), ("bf16x3", 1e-5)])
def test_cube_p2_64_galerkin_solve(precision, bar):
    p = cube_p2_64("galerkin", precision=precision)
    prob = K.Problem(K.desc_from_problem(p, seed=64))
    assert prob.N == 287496
    rc, lam, info = K.ka_eigs(prob.h, p["M"], tol=1e-5, maxit=80)
    prob.close()
    ref = product1d.galerkin_box_spectrum(p["p"], p["nel"], "gaussian", p["ell"], M=p["M"])
    err = errors.floored_rel_errors(ref, lam)
    print(p["name"], precision, info, "floored", err.max(), "raw", errors.rel_errors(ref, lam).max())
    assert rc == 0 and err.max() < bar


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-6), ("bf16x3", 1e-5)])
def test_cube_p2_64_collocation_solve(precision, bar):
    """Collocation on the 64^3 cube: 287,496 collocation rows x 7,077,888
    quadrature points (2.0e12 kernel pairs per block product, b = 64), against
    the exact product-of-1D collocation spectrum."""
    p = cube_p2_64("collocation", precision=precision)
    prob = K.Problem(K.desc_from_problem(p, seed=65))
    assert prob.N == 287496 and prob.Nquad == 7077888
    rc, lam, info = K.ka_eigs(prob.h, p["M"], tol=1e-5, maxit=80)
    prob.close()
    ref = product1d.collocation_box_spectrum(p["p"], p["nel"], "gaussian", p["ell"], M=p["M"])
    assert np.abs(ref.imag).max() == 0.0
    assert np.abs(lam[1::2]).max() <= 1e-6 * lam[0]
    err = errors.floored_rel_errors(ref.real, lam[0::2])
    print(p["name"], precision, info, "floored", err.max(), "raw", errors.rel_errors(ref.real, lam[0::2]).max())
    assert rc == 0 and err.max() < bar
