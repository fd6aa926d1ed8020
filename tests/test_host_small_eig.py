"""CPU unit tests of the library's small dense non-symmetric eigensolve
(Hessenberg reduction, eigenvalue QR on a banded copy, inverse iteration for
the wanted eigenvalues, back-transformation).  The same source runs on the GPU
inside ka_eigs for the collocation Rayleigh-Ritz step; here it is compiled for
the host with g++ and compared with LAPACK (numpy.linalg.eig).

The eigenvalue QR has two forms, both run here: double steps only (the
device's one-wave kernel below order 64), and multishift sweeps with a chain
of small bulges on large windows (the device's workgroup kernel from order
64), optionally moving the band to a second buffer part-way, as the device
moves it into LDS above order 196."""
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
    L.ka_host_nonsym_eig_ms.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_int]
    L.ka_host_nonsym_eig_ms.restype = ctypes.c_int
    L.ka_host_nonsym_values.argtypes = [dp, ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_int]
    L.ka_host_nonsym_values.restype = ctypes.c_int
    L.ka_host_ms_first_column.argtypes = [dp, ctypes.c_int] + [ctypes.c_double] * 4 + [dp]
    L.ka_host_pair_shifts.argtypes = [dp, dp, ctypes.c_int]
    return L


# QR forms: (multishift, order of the second band buffer or 0)
PATHS = {"double": (0, 0), "multishift": (1, 0), "multishift+move": (1, -1)}


def _eig(lib, H, nvec=None, path="double"):
    n = H.shape[0]
    nvec = n if nvec is None else nvec
    ms, fast = PATHS[path]
    if fast < 0:
        fast = n // 2 + 1          # the band moves once half the eigenvalues have deflated
    Hc = np.asfortranarray(H, dtype=np.float64)
    wr, wi, S = np.zeros(n), np.zeros(n), np.zeros((n, min(nvec + 1, n)), order="F")
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    nw = lib.ka_host_nonsym_eig_ms(p(Hc), n, nvec, p(wr), p(wi), p(S), ms, fast)
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


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("n", [1, 2, 3, 7, 40, 113, 200])
def test_random_nonsymmetric(lib, n, path):
    rng = np.random.default_rng(n)
    H = rng.standard_normal((n, n))
    nw, wr, wi, S = _eig(lib, H, path=path)
    assert nw == n
    _check(H, wr, wi, S, 1e-9)


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("n,nvec", [(5, 5), (64, 20), (150, 66), (196, 133), (228, 100)])
def test_nearly_symmetric_positive_spectrum(lib, n, nvec, path):
    # the Rayleigh-Ritz matrices of collocation: a small non-normal
    # perturbation of a symmetric positive matrix with decaying spectrum
    rng = np.random.default_rng(100 + n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = 0.5 ** (np.arange(n) / 8) + 1e-9
    H = (Q * lam) @ Q.T + 1e-6 * rng.standard_normal((n, n)) * lam[None, :]
    nw, wr, wi, S = _eig(lib, H, nvec, path=path)
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


def _values(lib, H, path):
    n = H.shape[0]
    ms, fast = PATHS[path]
    Hc = np.asfortranarray(H, dtype=np.float64)
    wr, wi = np.zeros(n), np.zeros(n)
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rc = lib.ka_host_nonsym_values(p(Hc), n, p(wr), p(wi), ms, n // 2 + 1 if fast < 0 else fast)
    return rc, wr + 1j * wi


def _match(lam, ref):
    # largest distance after pairing each computed eigenvalue with the nearest unused reference one
    used = np.zeros(ref.size, bool)
    err = 0.0
    for z in lam:
        d = np.abs(ref - z)
        d[used] = np.inf
        j = int(np.argmin(d))
        used[j] = True
        err = max(err, d[j])
    return err


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("n", [64, 229])
def test_cyclic_permutation_needs_exceptional_shifts(lib, n, path):
    # eigenvalues are the n-th roots of unity: all of one modulus, so the
    # standard shifts make no progress and only the exceptional ones help
    P = np.roll(np.eye(n), 1, axis=0)
    rc, lam = _values(lib, P, path)
    assert rc == 0
    assert np.allclose(np.abs(lam), 1.0, atol=1e-12)
    assert _match(lam, np.exp(2j * np.pi * np.arange(n) / n)) < 1e-12


@pytest.mark.parametrize("path", ["multishift", "multishift+move"])
@pytest.mark.parametrize("n", [100, 300])
def test_multishift_values_against_lapack(lib, n, path):
    # exactly six-fold clusters (cube symmetry) and conjugate pairs, hidden
    # by an orthogonal similarity
    rng = np.random.default_rng(40 + n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    for B in (np.diag(np.repeat(rng.uniform(0.1, 1.0, n // 6 + 1), 6)[:n]),
              np.diag(rng.uniform(-1, 1, n)) + np.diag(rng.uniform(0.2, 1, n - 1) * (np.arange(n - 1) % 2 == 0), 1)
              - np.diag(rng.uniform(0.2, 1, n - 1) * (np.arange(n - 1) % 2 == 0), -1)):
        H = Q @ B @ Q.T
        rc, lam = _values(lib, H, path)
        ref = np.linalg.eigvals(H)
        assert rc == 0
        assert _match(lam, ref) < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("shifts", [((0.3, 0.0), (-1.2, 0.0)), ((0.5, 0.7), (0.5, -0.7)), ((2.0, 0.0), (2.0, 0.0))])
def test_bulge_first_column_is_the_shift_polynomial(lib, shifts):
    # the bulge a shift pair introduces: the first column of
    # (H - s1 I)(H - s2 I), formed here as a matrix product
    rng = np.random.default_rng(11)
    n = 6
    H = np.triu(rng.standard_normal((n, n)), -1)
    (sr1, si1), (sr2, si2) = shifts
    v = np.zeros(3)
    lib.ka_host_ms_first_column(np.asfortranarray(H).ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n,
                                sr1, si1, sr2, si2, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    s1, s2 = complex(sr1, si1), complex(sr2, si2)
    ref = ((H - s1 * np.eye(n)) @ (H - s2 * np.eye(n)))[:, 0]
    assert np.abs(ref.imag).max() < 1e-12 and np.abs(ref[3:]).max() == 0.0
    ref = ref.real[:3]
    # equal up to a positive factor
    scale = np.dot(v, ref) / np.dot(v, v)
    assert scale > 0 and np.allclose(scale * v, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_shift_pairing(lib):
    # complex pairs stay together; real shifts pair up in descending order
    sr = np.array([0.1, 0.5, 0.5, -2.0, 3.0, 0.2, 0.2, 1.0])
    si = np.array([0.0, 0.4, -0.4, 0.0, 0.0, 1.5, -1.5, 0.0])
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    lib.ka_host_pair_shifts(p(sr), p(si), sr.size)
    assert list(zip(sr[:4], si[:4])) == [(0.5, 0.4), (0.5, -0.4), (0.2, 1.5), (0.2, -1.5)]
    assert list(sr[4:]) == [3.0, 1.0, 0.1, -2.0] and np.all(si[4:] == 0.0)
