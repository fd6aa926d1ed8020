"""CPU tests of the library's geometry evaluation (host_setup.cpp, run in
ka_setup): the general single-patch NURBS volume against the FP64 oracle's
independent evaluator and against finite differences of itself, the quarter
annulus given as a NURBS control net against its closed form, and the
rejection of invalid control nets."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import geometry
from workloads import nurbs_annulus_net, nurbs_blob_net

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "host", "geometry_host.cpp"),
       os.path.join(HERE, "..", "paper_2101_00629_amd", "csrc", "host_setup.cpp")]
INC = os.path.join(HERE, "..", "paper_2101_00629_amd", "csrc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("geo") / "libgeo_host.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", INC] + SRC + ["-o", so])
    L = ctypes.CDLL(so)
    L.ka_host_geometry_error.restype = ctypes.c_char_p
    return L


def _p(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _eval(lib, xh, net=None, ann=None):
    xh = np.ascontiguousarray(xh, dtype=np.float64)
    n = len(xh)
    x, J, W = np.zeros((n, 3)), np.zeros(n), np.zeros(n)
    if net is None:
        a = np.array(ann, dtype=np.float64)
        rc = lib.ka_host_geometry_eval(1, _p(a), None, None, None, None, n, _p(xh), _p(x), _p(J), _p(W))
    else:
        ctrl = np.ascontiguousarray(net["ctrl"], dtype=np.float64)
        deg = np.array(net["degree"], dtype=np.int32)
        nct = np.array([ctrl.shape[2], ctrl.shape[1], ctrl.shape[0]], dtype=np.int32)
        kn = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.float64) for t in net["knots"]]))
        rc = lib.ka_host_geometry_eval(2, None, _p(deg, ctypes.c_int), _p(nct, ctypes.c_int), _p(kn), _p(ctrl), n,
                                       _p(xh), _p(x), _p(J), _p(W))
    return rc, x, J, W


def _points(seed, n=400):
    xh = np.random.default_rng(seed).random((n, 3))
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=float)
    return np.vstack([corners, [[0.5, 0.0, 1.0], [1.0, 0.25, 0.0]], xh])


def test_annulus_net_matches_closed_form(lib):
    xh = _points(0)
    rc, x, J, W = _eval(lib, xh, net=nurbs_annulus_net(1.0, 2.0, 1.0))
    assert rc == 0
    rc2, x2, J2, _ = _eval(lib, xh, ann=(1.0, 2.0, 1.0))
    an = geometry.QuarterAnnulus()
    assert np.abs(x - an.map(xh)).max() < 1e-14 and np.abs(x2 - an.map(xh)).max() < 1e-14
    assert np.abs(J - an.detJ(xh)).max() < 1e-13 and np.abs(J2 - an.detJ(xh)).max() < 1e-13
    # the weight function is the quarter circle's denominator
    assert np.abs(W - geometry.circle_weight(xh[:, 0])).max() < 1e-15


@pytest.mark.parametrize("seed,degree,n", [(0, (2, 2, 2), (4, 4, 4)), (5, (3, 2, 1), (6, 3, 4)),
                                           (9, (1, 3, 2), (3, 5, 5))])
def test_nurbs_volume_matches_oracle(lib, seed, degree, n):
    net = nurbs_blob_net(seed, n=n, degree=degree)
    xh = _points(seed + 1)
    rc, x, J, W = _eval(lib, xh, net=net)
    assert rc == 0, lib.ka_host_geometry_error()
    o = geometry.NurbsVolume(net["degree"], net["knots"], net["ctrl"])
    xo, Jo, Wo = o._eval(xh)
    assert np.abs(x - xo).max() < 1e-14
    assert np.abs(J - np.abs(Jo)).max() < 1e-13 * np.abs(Jo).max()
    assert np.abs(W - Wo).max() < 1e-14
    assert J.min() > 0


def test_nurbs_jacobian_against_finite_differences(lib):
    net = nurbs_blob_net(2, n=(5, 4, 4), degree=(3, 2, 2))
    xh = 0.02 + 0.96 * np.random.default_rng(3).random((200, 3))     # interior: central differences
    h = 1e-6
    cols = []
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        cols.append((_eval(lib, xh + e, net=net)[1] - _eval(lib, xh - e, net=net)[1]) / (2 * h))
    dF = np.stack(cols, axis=-1)
    J = _eval(lib, xh, net=net)[2]
    assert np.abs(np.abs(np.linalg.det(dF)) - J).max() < 1e-7 * J.max()


def test_affine_net_is_the_identity(lib):
    # control points at the Greville abscissae with unit weights reproduce x = xh
    net = nurbs_blob_net(0, n=(5, 4, 6), degree=(3, 2, 2), wiggle=0.0, wrange=(1.0, 1.0))
    xh = _points(4)
    rc, x, J, W = _eval(lib, xh, net=net)
    assert rc == 0
    assert np.abs(x - xh).max() < 1e-14 and np.abs(J - 1).max() < 1e-13 and np.abs(W - 1).max() < 1e-15


def test_invalid_nets_are_rejected(lib):
    xh = _points(0, 4)
    good = nurbs_blob_net(1)
    bad_w = dict(good, ctrl=good["ctrl"].copy())
    bad_w["ctrl"][1, 2, 0, 3] = -0.5
    bad_open = dict(good, knots=([0, 0, 0.1, 0.5, 1, 1, 1],) + tuple(good["knots"][1:]))
    bad_order = dict(good, knots=([0, 0, 0, 0.7, 0.5, 1, 1, 1][:7],) + tuple(good["knots"][1:]))
    for net, word in ((bad_w, "weights"), (bad_open, "open"), (bad_order, "non-decreasing")):
        rc = _eval(lib, xh, net=net)[0]
        assert rc == -1 and word in lib.ka_host_geometry_error().decode()
