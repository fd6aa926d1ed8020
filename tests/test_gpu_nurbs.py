"""General single-patch NURBS volumes (domain KA_NURBS) on the GPU against
the FP64 oracle.

The curved test volume has weights drawn per control point, so they are not a
tensor product and Z is not a Kronecker product.  The oracle applies Z^-1 with
the complete-pivoting LU of the full Z (the paper's algorithm); the library
uses Z = diag(1/W(g)) (Z_3 x Z_2 x Z_1) instead.  Tolerances as in
test_gpu_operators: FP32 operator path 2e-5 (column-wise against max|ref|),
FP64 solves 1e-11, eigenvalues at the floored 1e-6 FP32 bar."""
import gc

import numpy as np
import pytest
import torch

import paper_2101_00629_amd as K
from oracle import collocation, errors, galerkin, geometry
from workloads import normal_block, nurbs_annulus_net, nurbs_blob_net

pytestmark = pytest.mark.gpu

BLOB = nurbs_blob_net(11, n=(5, 4, 4), degree=(3, 2, 2), wiggle=0.05)

CASES = [
    dict(method="collocation", p=2, nel=(4, 3, 5), kernel="gaussian", ell=0.5),
    dict(method="collocation", p=3, nel=(3, 4, 2), kernel="exponential", ell=0.7, sigma=1.3),
    dict(method="galerkin", p=2, nel=(4, 3, 5), kernel="exponential", ell=1.0),
    dict(method="galerkin", p=3, nel=(3, 4, 2), kernel="gaussian", ell=0.5),
    dict(method="galerkin_gauss", p=2, nel=(3, 2, 2), kernel="gaussian", ell=0.5, sigma=0.8),
]


def _ids(c):
    return f"{c['method']}-p{c['p']}-{c['kernel']}"


def _oracle(c, net=BLOB):
    dom = geometry.NurbsVolume(net["degree"], net["knots"], net["ctrl"])
    cls = {"collocation": collocation.Collocation, "galerkin": galerkin.GalerkinIBQ,
           "galerkin_gauss": galerkin.GalerkinGauss}[c["method"]]
    return cls(dom, c["p"], c["nel"], c["kernel"], c["ell"], c.get("sigma", 1.0))


def _problem(c, net=BLOB, **kw):
    return K.Problem(K.make_desc(domain="nurbs", nurbs=net, **c, **kw))


def _gpu_apply(prob, form, X):
    Xd = torch.tensor(X.T.copy(), dtype=torch.float64, device="cuda")
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
    X = normal_block(31, o.N, 20)           # two passes of b = 16, the second ragged
    for form in (K.KA_A, K.KA_APRIME):
        Y = _gpu_apply(prob, form, X)
        ref = o.apply_A(X) if form == K.KA_A else o.apply_Aprime(X)
        err, tol = _colerr(Y, ref), 2e-5
        if form == K.KA_APRIME and c["method"] == "collocation":
            # backward error Z Y - A X at the FP32 bar; forward error up to cond(Z)
            back = _colerr(o.Z_dense() @ Y, o.apply_A(X))
            assert back < 2e-5, back
            tol *= np.linalg.cond(o.Z_dense())
        assert np.isfinite(Y).all() and err < tol, (form, err, tol)
    prob.close()


def test_zinv_matches_complete_pivot_lu():
    c = CASES[1]
    o = _oracle(c)
    prob = _problem(c)
    X = normal_block(32, o.N, 9)
    Xd = torch.tensor(X.T.copy(), dtype=torch.float64, device="cuda")
    K.ka_solve_Z(prob.h, K.KA_ZINV, Xd)
    torch.cuda.synchronize()
    ref = o.solve_Z(X)
    assert np.abs(Xd.cpu().numpy().T - ref).max() < 1e-11 * np.abs(ref).max()
    prob.close()


@pytest.mark.parametrize("method,kernel,ell", [("collocation", "gaussian", 0.5), ("collocation", "exponential", 0.8),
                                               ("galerkin", "gaussian", 0.5), ("galerkin", "exponential", 1.0)])
def test_eigenvalues_match_oracle(method, kernel, ell):
    c = dict(method=method, p=2, nel=(4, 3, 4), kernel=kernel, ell=ell)
    o = _oracle(c)
    ref, _ = o.eig_dense()
    prob = _problem(c, seed=5)
    M = 12
    rc, lam, info = K.ka_eigs(prob.h, M, tol=1e-6, maxit=80)
    prob.close()
    assert rc == 0
    if method == "collocation":
        assert np.abs(lam[1::2]).max() <= 1e-6 * lam[0]
        lam, ref = lam[0::2], ref.real
    err = errors.floored_rel_errors(ref[:M], lam[:M])
    print(method, kernel, info, "floored", err.max())
    assert err.max() < 1e-6


@pytest.mark.parametrize("method", ["collocation", "galerkin"])
def test_annulus_net_matches_closed_form_domain(method):
    """The quarter annulus given as a control net (rational basis B_j / W,
    row and column scales W) against the closed-form domain (tensor weights
    folded into the univariate factors): the same spectrum."""
    c = dict(method=method, p=3, nel=(8, 8, 4), kernel="exponential", ell=0.5, block=16)
    M = 20
    lams = []
    for desc in (K.make_desc(domain="quarter_annulus", seed=9, **c),
                 K.make_desc(domain="nurbs", nurbs=nurbs_annulus_net(), seed=9, **c)):
        prob = K.Problem(desc)
        rc, lam, info = K.ka_eigs(prob.h, M, tol=1e-6, maxit=80)
        prob.close()
        assert rc == 0
        lams.append(lam[0::2] if method == "collocation" else lam)
    err = errors.floored_rel_errors(lams[0], lams[1])
    print(method, "closed form vs control net, floored", err.max())
    assert err.max() < 1e-6


def test_server_copies_the_control_net():
    c = dict(method="collocation", p=2, nel=(4, 3, 4), kernel="gaussian", ell=0.5, block=16)
    M = 10
    prob = _problem(c, seed=21)
    rc, ref, _ = K.ka_eigs(prob.h, M, tol=1e-6, maxit=80)
    prob.close()
    assert rc == 0
    net = {k: (np.array(v, copy=True) if k == "ctrl" else tuple(np.array(t, dtype=float) for t in v)
               if k == "knots" else v) for k, v in BLOB.items()}
    desc = K.make_desc(domain="nurbs", nurbs=net, seed=21, **c)
    srv = K.ka_server_create(8 << 30, 2)
    lam = np.zeros(2 * M)
    K.ka_server_submit(srv, desc, M, lam, tol=1e-6, maxit=80, arrival_s=0.0, tag=0)
    for a in desc._keep:            # the caller's arrays change after submit
        a[...] = np.nan
    del desc, net
    gc.collect()
    K.ka_server_run(srv, 120.0)
    res = K.ka_server_poll(srv)
    K.ka_server_destroy(srv)
    assert res[0]["status"] == 0
    assert np.abs(lam[0::2] - ref[0::2]).max() <= 1e-6 * abs(ref[0])

