"""CPU unit tests of the library's small dense non-symmetric eigensolve
(Hessenberg reduction, eigenvalue QR on a banded copy, inverse iteration for
the wanted eigenvalues, back-transformation).  The same source runs on the GPU
inside ka_eigs for the collocation Rayleigh-Ritz step; here it is compiled for
the host with g++ and compared with LAPACK (numpy.linalg.eig)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "nonsym_host.cpp")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("nonsym") / "libnonsym_host.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", SRC, "-o", so])
    L = ctypes.CDLL(so)
    dp = ctypes.POINTER(ctypes.c_double)
    L.ka_host_nonsym_eig.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp, dp]
    L.ka_host_nonsym_eig.restype = ctypes.c_int
    return L


def _eig(lib, H, nvec=None):
    n = H.shape[0]
    nvec = n if nvec is None else nvec
    Hc = np.asfortranarray(H, dtype=np.float64)
    wr, wi, S = np.zeros(n), np.zeros(n), np.zeros((n, min(nvec + 1, n)), order="F")
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    nw = lib.ka_host_nonsym_eig(p(Hc), n, nvec, p(wr), p(wi), p(S))
    return nw, wr, wi, S[:, :max(nw, 0)]


def _check(H, wr, wi, S, tol):
    n = H.shape[0]
    lam = wr + 1j * wi
    assert np.all(np.diff(wr) <= 1e-12 * np.abs(wr).max())      # descending real part
    ref = np.linalg.eigvals(H)
    assert np.allclose(np.sort_complex(lam), np.sort_complex(ref), atol=tol * np.abs(ref).max())
    scale = np.abs(H).max()
    j = 0
    while j < S.shape[1]:
        if wi[j] == 0:
            v = S[:, j]
            assert abs(np.linalg.norm(v) - 1) < 1e-10
            assert np.linalg.norm(H @ v - wr[j] * v) < tol * scale, j
            j += 1
        else:
            assert wi[j] > 0 and wi[j + 1] == -wi[j]
            v = S[:, j] + 1j * S[:, j + 1]
            assert abs(np.linalg.norm(v) - 1) < 1e-10
            assert np.linalg.norm(H @ v - lam[j] * v) < tol * scale, j
            j += 2


@pytest.mark.parametrize("n", [1, 2, 3, 7, 40, 113, 200])
def test_random_nonsymmetric(lib, n):
    rng = np.random.default_rng(n)
    H = rng.standard_normal((n, n))
    nw, wr, wi, S = _eig(lib, H)
    assert nw == n
    _check(H, wr, wi, S, 1e-9)


@pytest.mark.parametrize("n,nvec", [(5, 5), (64, 20), (150, 66), (196, 133)])
def test_nearly_symmetric_positive_spectrum(lib, n, nvec):
    # the Rayleigh-Ritz matrices of collocation: a small non-normal
    # perturbation of a symmetric positive matrix with decaying spectrum
    rng = np.random.default_rng(100 + n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = 0.5 ** (np.arange(n) / 8) + 1e-9
    H = (Q * lam) @ Q.T + 1e-6 * rng.standard_normal((n, n)) * lam[None, :]
    nw, wr, wi, S = _eig(lib, H, nvec)
    assert nw in (nvec, nvec + 1)
    _check(H, wr, wi, S, 1e-9)
    assert np.allclose(wr[:10], np.sort(np.linalg.eigvals(H).real)[::-1][:10], rtol=1e-9)


def test_rotation_blocks_and_complex_pairs(lib):
    # block diagonal with explicit 2x2 rotation blocks (complex pairs) and
    # repeated real eigenvalues, hidden by an orthogonal similarity
    rng = np.random.default_rng(7)
    B = np.zeros((9, 9))
    B[0:2, 0:2] = [[1.0, -2.0], [2.0, 1.0]]
    B[2:4, 2:4] = [[0.3, 0.5], [-0.5, 0.3]]
    B[4, 4] = B[5, 5] = 2.0
    B[6, 6], B[7, 7], B[8, 8] = -1.0, 0.0, 0.5
    B[4, 6] = 0.3
    Q, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    H = Q @ B @ Q.T
    nw, wr, wi, S = _eig(lib, H)
    _check(H, wr, wi, S, 1e-8)
    assert np.sum(wi != 0) == 4
    # a pair straddling the wanted count is kept whole
    nw, wr, wi, S = _eig(lib, H, nvec=2)
    assert wr[0] == 2.0 or wi[1] != 0 or nw >= 2


def test_degenerate_cluster_gives_independent_vectors(lib):
    # cube symmetry: triple and six-fold eigenvalues of a symmetric matrix
    rng = np.random.default_rng(3)
    lam = np.array([1.0, 0.5, 0.5, 0.5, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25, 0.1, 0.05])
    n = lam.size
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    H = (Q * lam) @ Q.T
    nw, wr, wi, S = _eig(lib, H, nvec=10)
    _check(H, wr, wi, S, 1e-9)
    assert np.linalg.svd(S, compute_uv=False).min() > 0.5   # a basis of each eigenspace


def test_symmetric_input(lib):
    rng = np.random.default_rng(9)
    A = rng.standard_normal((30, 30))
    H = A + A.T
    nw, wr, wi, S = _eig(lib, H)
    assert np.all(wi == 0)
    _check(H, wr, wi, S, 1e-9)
    assert np.allclose(wr, np.sort(np.linalg.eigvalsh(H))[::-1], atol=1e-10 * np.abs(H).max())
