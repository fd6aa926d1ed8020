"""Parity of the matrix-free operators (ka_apply_A) and the Kronecker solves
(ka_solve_Z) with the FP64 oracle, on meshes that span several tiles and
ragged tails, on the cube and the curved quarter annulus.

The operator path computes the transfers and the kernel product in FP32, so
results are compared column-wise against max|ref| with tol = 2e-5 (FP32 unit
roundoff times the short chains of the Kronecker transfers and the kernel
sum).  The solves are pure FP64: tol = 1e-12.
"""
import numpy as np
import pytest
import torch

import paper_2101_00629_amd as K
from oracle import collocation, galerkin, geometry
from workloads import normal_block

pytestmark = pytest.mark.gpu

CASES = [
    dict(method="galerkin", domain="cube", p=2, nel=(4, 3, 5), kernel="exponential", ell=1.0),
    dict(method="galerkin", domain="quarter_annulus", p=3, nel=(3, 4, 2), kernel="gaussian", ell=0.5),
    dict(method="galerkin", domain="cube", p=3, nel=(5, 4, 3), kernel="gaussian", ell=0.3, sigma=1.7),
    dict(method="collocation", domain="cube", p=2, nel=(4, 3, 5), kernel="gaussian", ell=0.5),
    dict(method="collocation", domain="quarter_annulus", p=3, nel=(3, 4, 2), kernel="exponential", ell=0.7),
    dict(method="collocation", domain="quarter_annulus", p=4, nel=(4, 2, 3), kernel="gaussian", ell=0.5,
         sigma=0.8),
    dict(method="galerkin_gauss", domain="cube", p=2, nel=(4, 3, 5), kernel="exponential", ell=1.0),
    dict(method="galerkin_gauss", domain="quarter_annulus", p=3, nel=(3, 2, 2), kernel="gaussian", ell=0.5,
         sigma=1.3),
]


def _ids(c):
    return f"{c['method']}-{c['domain']}-p{c['p']}-{c['kernel']}"


def _oracle(c):
    dom = geometry.make_domain(c["domain"])
    if c["method"] == "galerkin_gauss":
        return galerkin.GalerkinGauss(dom, c["p"], c["nel"], c["kernel"], c["ell"], c.get("sigma", 1.0))
    if c["method"] == "galerkin":
        return galerkin.GalerkinIBQ(dom, c["p"], c["nel"], c["kernel"], c["ell"], c.get("sigma", 1.0))
    return collocation.Collocation(dom, c["p"], c["nel"], c["kernel"], c["ell"], c.get("sigma", 1.0))


def _problem(c, block=16, precision="fp32"):
    return K.Problem(K.make_desc(block=block, precision=precision, **c))


def _gpu_apply(prob, form, X):
    Xd = torch.tensor(X.T.copy(), dtype=torch.float64, device="cuda")    # (nvec, N): column-major block
    Yd = torch.full_like(Xd, float("nan"))
    K.ka_apply_A(prob.h, form, Xd, Yd)
    torch.cuda.synchronize()
    return Yd.cpu().numpy().T


def _colerr(Y, ref):
    return (np.abs(Y - ref).max(axis=0) / np.abs(ref).max(axis=0)).max()


@pytest.mark.parametrize("c", CASES, ids=_ids)
def test_apply_matches_oracle(c):
    o = _oracle(c)
    prob = _problem(c)
    assert prob.N == o.N
    X = normal_block(21, o.N, 20)          # 20 > block: two passes, the second ragged
    for form in (K.KA_A, K.KA_APRIME):
        Y = _gpu_apply(prob, form, X)
        ref = o.apply_A(X) if form == K.KA_A else o.apply_Aprime(X)
        err = _colerr(Y, ref)
        tol = 2e-5
        if form == K.KA_APRIME and c["method"] == "collocation":
            # A' = Z^-1 A: the FP64 solve is exact, but it amplifies the FP32
            # error of A X by up to cond(Z) = prod_k cond(Z_k).  Check the
            # backward error Z Y - A X at the FP32 bar and the forward error
            # against the condition number.
            AX = o.apply_A(X)
            back = _colerr(o.Z_dense() @ Y, AX)
            assert back < 2e-5, back
            tol *= np.prod([np.linalg.cond(Zk) for Zk in o.Zk])
        assert np.isfinite(Y).all() and err < tol, (form, err, tol)
    prob.close()


@pytest.mark.parametrize("c", [CASES[1], CASES[4]], ids=_ids)
def test_apply_bf16x3(c):
    o = _oracle(c)
    prob = _problem(c, precision="bf16x3")
    X = normal_block(22, o.N, 16)
    Y = _gpu_apply(prob, K.KA_APRIME, X)
    assert _colerr(Y, o.apply_Aprime(X)) < 2e-4
    prob.close()


@pytest.mark.parametrize("c", [CASES[0], CASES[1], CASES[4]], ids=_ids)
def test_solves_match_oracle(c):
    o = _oracle(c)
    prob = _problem(c)
    X = normal_block(23, o.N, 7)
    ops = [(K.KA_ZINV, o.solve_Z(X))]
    if c["method"] == "galerkin":
        ops.append((K.KA_LINV, o._Lsolve(X, trans=0)))
        ops.append((K.KA_LTINV, o._Lsolve(X, trans=1)))
    for op, ref in ops:
        Xd = torch.tensor(X.T.copy(), dtype=torch.float64, device="cuda")
        K.ka_solve_Z(prob.h, op, Xd)
        torch.cuda.synchronize()
        got = Xd.cpu().numpy().T
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max(), op
    if c["method"] == "collocation":
        with pytest.raises(K.KAError):
            K.ka_solve_Z(prob.h, K.KA_LINV, torch.zeros((1, prob.N), dtype=torch.float64, device="cuda"))
    prob.close()


def test_dense_columns_brute_force():
    # apply A to every unit vector of a tiny problem and compare entrywise with
    # the densely assembled oracle matrices
    for c in (dict(method="galerkin", domain="quarter_annulus", p=2, nel=(2, 3, 2), kernel="exponential", ell=0.6),
              dict(method="collocation", domain="cube", p=2, nel=(2, 2, 3), kernel="gaussian", ell=0.4)):
        o = _oracle(c)
        prob = _problem(c)
        E = np.eye(o.N)
        A = _gpu_apply(prob, K.KA_A, E)
        ref = o.A_dense()
        assert np.abs(A - ref).max() < 2e-5 * np.abs(ref).max()
        Ap = _gpu_apply(prob, K.KA_APRIME, E)
        if c["method"] == "galerkin":
            L = np.linalg.cholesky(o.Z_dense())
            refp = np.linalg.solve(L, np.linalg.solve(L, ref).T).T
        else:
            refp = o.Aprime_dense()
        assert np.abs(Ap - refp).max() < 2e-5 * np.abs(refp).max()
        prob.close()


def test_galerkin_operator_symmetric():
    c = CASES[1]
    prob = _problem(c)
    X = normal_block(24, prob.N, 16)
    AX = _gpu_apply(prob, K.KA_APRIME, X)
    G = X.T @ AX
    assert np.abs(G - G.T).max() < 1e-5 * np.abs(G).max()
    assert np.linalg.eigvalsh(0.5 * (G + G.T)).min() > -1e-5 * np.abs(G).max()
    prob.close()
