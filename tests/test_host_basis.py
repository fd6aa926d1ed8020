"""CPU unit tests of the library's restart basis: diagonal-pivoted Cholesky of
the Gram matrix G = S^T S of the kept Ritz vectors, with a rank cut, giving W
with S W orthonormal.  The same source runs on the GPU inside ka_eigs for the
thick restart of the collocation (non-symmetric) eigensolver; here it is
compiled for the host with g++ and checked against what a basis of span(S) must
satisfy, and against numpy's Cholesky on a full-rank case."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "basis_host.cpp")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("basis") / "libbasis_host.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", SRC, "-o", so])
    L = ctypes.CDLL(so)
    dp = ctypes.POINTER(ctypes.c_double)
    L.ka_host_pchol_basis.argtypes = [dp, ctypes.c_int, ctypes.c_double, dp]
    L.ka_host_pchol_basis.restype = ctypes.c_int
    return L


def _basis(lib, S, cut=1e-12):
    G = np.asfortranarray(S.T @ S)
    n = G.shape[0]
    W = np.full((n, n), np.nan, order="F")
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    r = lib.ka_host_pchol_basis(p(G), n, cut, p(W))
    return r, W[:, :r]


def _span_check(S, Q, tol):
    # every column of S lies in span(Q), and Q lies in span(S)
    res = S - Q @ (Q.T @ S)
    assert np.linalg.norm(res) <= tol * np.linalg.norm(S)
    U, sv, _ = np.linalg.svd(S, full_matrices=False)
    U = U[:, sv > 1e-10 * sv[0]]
    assert np.linalg.norm(Q - U @ (U.T @ Q)) <= tol * np.sqrt(Q.shape[1])


@pytest.mark.parametrize("k,n", [(40, 10), (120, 60), (300, 133)])
def test_full_rank_gives_orthonormal_basis_of_the_span(lib, k, n):
    rng = np.random.default_rng(k + n)
    S = rng.standard_normal((k, n))
    S /= np.linalg.norm(S, axis=0)
    r, W = _basis(lib, S)
    assert r == n
    Q = S @ W
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-12
    _span_check(S, Q, 1e-12)


def test_matches_cholesky_of_the_pivoted_gram(lib):
    # W = P R^-1 with P^T G P = R^T R: R from numpy's Cholesky of the permuted
    # G, the permutation read from W's structure (row piv[i] of W is the last
    # nonzero of column i)
    rng = np.random.default_rng(3)
    S = rng.standard_normal((50, 12)) * rng.uniform(0.5, 3.0, 12)
    r, W = _basis(lib, S)
    assert r == 12
    order = []
    for i in range(r):
        nz = set(np.flatnonzero(np.abs(W[:, i]) > 0)) - set(order)
        assert len(nz) == 1
        order.append(nz.pop())
    P = np.eye(12)[:, order]
    R = np.linalg.cholesky(P.T @ (S.T @ S) @ P).T
    assert np.allclose(P.T @ W, np.linalg.inv(R), rtol=1e-10, atol=1e-12)
    # diagonal pivoting: the first pivot is the longest column
    assert order[0] == int(np.argmax(np.linalg.norm(S, axis=0)))


def test_dependent_columns_are_cut(lib):
    rng = np.random.default_rng(7)
    A = rng.standard_normal((80, 9))
    S = np.hstack([A, A @ rng.standard_normal((9, 5))])   # 14 columns of rank 9
    S = S[:, rng.permutation(14)]
    r, W = _basis(lib, S)
    assert r == 9
    Q = S @ W
    assert np.abs(Q.T @ Q - np.eye(r)).max() < 1e-9
    _span_check(S, Q, 1e-9)


def test_nearly_dependent_column_is_cut_at_the_threshold(lib):
    rng = np.random.default_rng(11)
    A = rng.standard_normal((60, 6))
    A /= np.linalg.norm(A, axis=0)
    extra = A @ rng.standard_normal(6)
    extra /= np.linalg.norm(extra)
    e = rng.standard_normal(60)
    e -= A @ np.linalg.lstsq(A, e, rcond=None)[0]
    e /= np.linalg.norm(e)
    for dist, kept in ((1e-3, 7), (1e-8, 6)):
        S = np.hstack([A, (extra + dist * e)[:, None]])
        r, _ = _basis(lib, S, cut=1e-12)
        assert r == kept, (dist, r)


def test_zero_and_single(lib):
    r, _ = _basis(lib, np.zeros((10, 4)))
    assert r == 0
    s = np.arange(1.0, 6.0)[:, None]
    r, W = _basis(lib, s)
    assert r == 1 and abs(W[0, 0] - 1.0 / np.linalg.norm(s)) < 1e-15
