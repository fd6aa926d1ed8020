"""CPU unit tests of the library's small dense symmetric eigensolve
(Householder tridiagonalisation, bisection, inverse iteration with cluster
orthogonalisation, back-transformation).  The same source runs on the GPU
inside ka_eigs for the Galerkin Rayleigh-Ritz step; here it is compiled for
the host with g++ and compared with LAPACK (numpy.linalg.eigh)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "sym_host.cpp")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("sym") / "libsym_host.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", SRC, "-o", so])
    L = ctypes.CDLL(so)
    dp = ctypes.POINTER(ctypes.c_double)
    L.ka_host_sym_eig.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp]
    L.ka_host_sym_eig.restype = ctypes.c_int
    L.ka_host_sym_eig_nb.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int]
    L.ka_host_sym_eig_nb.restype = ctypes.c_int
    return L


def _eig(lib, H, nvec=None):
    n = H.shape[0]
    nvec = n if nvec is None else nvec
    Hc = np.asfortranarray(H, dtype=np.float64)
    th, S = np.zeros(n), np.zeros((n, nvec), order="F")
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    nc = lib.ka_host_sym_eig(p(Hc), n, nvec, p(th), p(S))
    return nc, th, S


def _check(H, th, S, tol=1e-12):
    n = H.shape[0]
    nvec = S.shape[1]
    scale = max(np.abs(np.linalg.eigvalsh(H)).max(), 1e-300)
    ref = np.sort(np.linalg.eigvalsh(H))[::-1]
    assert np.all(np.diff(th) <= 0)
    assert np.abs(th - ref).max() <= tol * scale * max(1, n / 10)
    # residuals and orthonormality of the computed vectors
    R = H @ S - S * th[None, :nvec]
    assert np.linalg.norm(R, axis=0).max() <= 100 * tol * scale * np.sqrt(n)
    assert np.abs(S.T @ S - np.eye(nvec)).max() <= 1e-10


@pytest.mark.parametrize("n", [1, 2, 3, 8, 37, 114, 228])
def test_random_symmetric(lib, n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    H = A + A.T
    nc, th, S = _eig(lib, H)
    _check(H, th, S)


@pytest.mark.parametrize("n", [20, 120])
def test_decaying_positive_spectrum(lib, n):
    # Rayleigh-Ritz matrices of the K-L operator: positive, fast decay
    rng = np.random.default_rng(50 + n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = 0.7 ** np.arange(n)
    H = (Q * lam) @ Q.T
    nc, th, S = _eig(lib, H)
    _check(H, th, S)
    assert np.allclose(th[:20], lam[:20], rtol=1e-10, atol=1e-14)


def test_exact_multiplicities(lib):
    # cube symmetry gives repeated eigenvalues; hide them by a rotation
    rng = np.random.default_rng(3)
    lam = np.array([1.0, 0.5, 0.5, 0.5, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25, 0.1, 0.0, 0.0, -0.3])
    n = lam.size
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    H = (Q * lam) @ Q.T
    nc, th, S = _eig(lib, H)
    _check(H, th, S)
    assert nc == 6       # clusters {1}, {.5 x3}, {.25 x6}, {.1}, {0 x2}, {-.3}
    # leading vectors only; the cut falls inside the six-fold cluster
    nc, th, S = _eig(lib, H, nvec=7)
    _check(H, th, S)
    assert nc == 3


def test_near_degenerate_and_tiny(lib):
    # pairs split by 1e-9 (one cluster each), a tail of tiny eigenvalues
    rng = np.random.default_rng(4)
    lam = np.concatenate([[1.0, 1.0 - 1e-9, 0.6, 0.6 + 3e-7, 0.3], 1e-14 * rng.random(40)])
    n = lam.size
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    H = (Q * lam) @ Q.T
    nc, th, S = _eig(lib, H)
    _check(H, th, S)


def test_already_tridiagonal_and_diagonal(lib):
    n = 50
    H = np.diag(np.arange(n, 0, -1.0)) + np.diag(np.full(n - 1, 0.5), 1) + np.diag(np.full(n - 1, 0.5), -1)
    nc, th, S = _eig(lib, H)
    _check(H, th, S)
    D = np.diag(np.linspace(2, -1, 33))
    nc, th, S = _eig(lib, D)
    _check(D, th, S)
    Z = np.zeros((5, 5))
    nc, th, S = _eig(lib, Z)
    assert np.abs(th).max() < 1e-15 and np.abs(S.T @ S - np.eye(5)).max() < 1e-12


@pytest.mark.parametrize("nvec", [1, 10, 66])
def test_leading_vectors_only(lib, nvec):
    # Rayleigh-Ritz use: all eigenvalues, the leading nvec vectors, a tail of
    # numerically zero eigenvalues that is never touched
    rng = np.random.default_rng(11)
    n = 114
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([0.9 ** np.arange(70), 1e-17 * rng.random(n - 70)])
    H = (Q * lam) @ Q.T
    nc, th, S = _eig(lib, H, nvec=nvec)
    _check(H, th, S)


def _eig_nb(lib, H, nb, nvec=None):
    n = H.shape[0]
    nvec = n if nvec is None else nvec
    Hc = np.asfortranarray(H, dtype=np.float64)
    th, S = np.zeros(n), np.zeros((n, nvec), order="F")
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    nc = lib.ka_host_sym_eig_nb(p(Hc), n, nvec, p(th), p(S), nb)
    return nc, th, S


@pytest.mark.parametrize("nb", [1, 3, 8])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 9, 10, 11, 37, 130, 229])
def test_blocked_tridiagonalisation(lib, n, nb):
    """The blocked reduction (deferred panel updates) against LAPACK, on panel
    counts that divide n - 2 and ones that leave a ragged last panel; its
    eigenvalues also match the unblocked reduction's to rounding."""
    rng = np.random.default_rng(1000 + n)
    A = rng.standard_normal((n, n))
    H = A + A.T
    nc, th, S = _eig_nb(lib, H, nb)
    _check(H, th, S)
    _, th0, _ = _eig(lib, H)
    assert np.abs(th - th0).max() <= 1e-12 * max(np.abs(th0).max(), 1e-300) * max(1, n / 10)


@pytest.mark.parametrize("nb", [3, 8])
def test_blocked_multiplicities_and_zero_columns(lib, nb):
    # exact multiplicities (zero reflectors: columns already reduced) and a
    # matrix with an exactly zero off-diagonal block
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((40, 40)))
    lam = np.repeat([3.0, 1.0, -2.0, 0.5], 10)
    H = (Q * lam) @ Q.T
    nc, th, S = _eig_nb(lib, H, nb)
    _check(H, th, S)
    B = np.zeros((24, 24))
    B[:12, :12] = np.diag(np.arange(12.0))
    B[12:, 12:] = np.eye(12) * 2.0 + 0.1
    nc, th, S = _eig_nb(lib, B, nb)
    _check(B, th, S)
