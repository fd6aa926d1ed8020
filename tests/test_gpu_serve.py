"""Continuous-batching server: admission by device footprint, arrivals while
others run, and results that are the same alone and in the mix (bitwise
between server runs; within FP32 rounding of the plain single-problem solve,
which launches the single-product kernel instead of the batched one)."""
import numpy as np
import pytest
import torch

import paper_2101_00629_amd as K
from oracle import errors, product1d

pytestmark = pytest.mark.gpu

MIX = [
    dict(method="galerkin", domain="cube", p=2, nel=(6, 6, 6), kernel="exponential", ell=1.0, M=10, block=16),
    dict(method="collocation", domain="cube", p=3, nel=(5, 5, 5), kernel="gaussian", ell=0.5, M=12, block=16),
    dict(method="galerkin", domain="quarter_annulus", p=3, nel=(6, 6, 3), kernel="gaussian", ell=0.7, M=20,
         block=32),
    dict(method="collocation", domain="quarter_annulus", p=2, nel=(6, 5, 3), kernel="exponential", ell=0.4, M=8,
         block=16),
    dict(method="galerkin", domain="cube", p=3, nel=(7, 7, 7), kernel="gaussian", ell=0.3, M=30, block=32,
         precision="bf16x3"),
    dict(method="galerkin", domain="cube", p=2, nel=(8, 8, 8), kernel="gaussian", ell=0.5, M=16, block=16),
]
ARRIVALS = [0.0, 0.0, 0.005, 0.01, 0.02, 0.03]


def _desc(c, i):
    c = dict(c)
    c.pop("M")
    return K.make_desc(seed=100 + i, **c)


def _serve(cases, arrivals, budget=8 << 30, slots=8):
    srv = K.ka_server_create(budget, slots)
    lams = []
    for i, (c, t) in enumerate(zip(cases, arrivals)):
        lam = np.zeros(2 * c["M"])
        lams.append(lam)
        K.ka_server_submit(srv, _desc(c, i), c["M"], lam, tol=1e-5, maxit=60, arrival_s=t, tag=i)
    K.ka_server_run(srv, 120.0)
    res = sorted(K.ka_server_poll(srv), key=lambda r: r["tag"])
    stats = K.ka_server_stats(srv)
    K.ka_server_destroy(srv)
    return lams, res, stats


def _plain(c, i):
    prob = K.Problem(_desc(c, i))
    rc, lam, info = K.ka_eigs(prob.h, c["M"], tol=1e-5, maxit=60)
    prob.close()
    return rc, lam


def test_mix_equals_alone_and_plain():
    lam_mix, res, stats = _serve(MIX, ARRIVALS)
    assert len(res) == len(MIX) and all(r["status"] == 0 for r in res), res
    assert stats["max_active"] >= 3                 # requests overlapped on the device
    assert stats["bytes_in_use"] == 0               # every arena range returned
    for i, c in enumerate(MIX):
        lam_alone, res1, _ = _serve_single(c, i)      # same seed as in the mix
        n = c["M"] * (2 if c["method"] == "collocation" else 1)
        assert np.array_equal(lam_mix[i][:n], lam_alone[:n]), (i, lam_mix[i][:n] - lam_alone[:n])
        rc, lam_p = _plain(c, i)
        assert rc == 0
        ref = lam_p[0::2] if c["method"] == "collocation" else lam_p
        got = lam_mix[i][:n][0::2] if c["method"] == "collocation" else lam_mix[i][:n]
        assert np.abs(got - ref).max() <= 1e-6 * abs(ref[0]), (i, np.abs(got - ref).max())


def _serve_single(c, i):
    srv = K.ka_server_create(8 << 30, 1)
    lam = np.zeros(2 * c["M"])
    K.ka_server_submit(srv, _desc(c, i), c["M"], lam, tol=1e-5, maxit=60, arrival_s=0.0, tag=i)
    K.ka_server_run(srv, 120.0)
    res = K.ka_server_poll(srv)
    K.ka_server_destroy(srv)
    assert res[0]["status"] == 0
    return lam, res, None


def test_served_eigenvalues_match_oracle():
    c = MIX[5]
    lam, res, _ = _serve([c], [0.0])
    ref = product1d.galerkin_box_spectrum(2, (8, 8, 8), "gaussian", 0.5, M=c["M"])
    assert errors.floored_rel_errors(ref, lam[0][:c["M"]]).max() < 1e-6


def test_admission_by_memory_budget():
    cases = [MIX[5], MIX[5], MIX[5], MIX[5]]
    need = [K.ka_request_bytes(_desc(c, i), c["M"]) for i, c in enumerate(cases)]
    # room for one request at a time, not two: they run one after the other
    lam, res, stats = _serve(cases, [0.0] * 4, budget=int(1.5 * max(need)), slots=4)
    assert all(r["status"] == 0 for r in res)
    assert stats["max_active"] == 1
    # room for two at a time
    lam, res, stats = _serve(cases, [0.0] * 4, budget=int(2.5 * max(need)), slots=4)
    assert all(r["status"] == 0 for r in res) and stats["max_active"] == 2
    # a request that can never fit is rejected with KA_ERR_OOM, the rest still run
    small = K.ka_request_bytes(_desc(MIX[0], 0), MIX[0]["M"])
    lam, res, stats = _serve([MIX[0], MIX[2]], [0.0, 0.0], budget=int(1.1 * small), slots=4)
    st = {r["tag"]: r["status"] for r in res}
    assert st[0] == 0 and st[1] == K.KA_ERR_OOM


def test_late_arrivals_join_running_batch():
    big = dict(method="galerkin", domain="quarter_annulus", p=3, nel=(14, 14, 7), kernel="exponential", ell=0.5,
               M=40, block=32)
    cases = [big, MIX[0], MIX[1]]
    lam, res, stats = _serve(cases, [0.0, 0.002, 0.004], slots=8)
    assert all(r["status"] == 0 for r in res)
    by = {r["tag"]: r for r in res}
    # a later request was admitted before the first one finished
    assert by[1]["admit_s"] < by[0]["done_s"] or by[2]["admit_s"] < by[0]["done_s"]
    for r in res:
        assert r["admit_s"] >= r["arrival_s"] - 1e-9 and r["done_s"] >= r["admit_s"]
