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
        rc = lib.ka_host_geometry_eval(1, _p(a), None, None, None, None, n, _p(xh), _p(x), _p(J), _p(W), None)
    else:
        ctrl = np.ascontiguousarray(net["ctrl"], dtype=np.float64)
        deg = np.array(net["degree"], dtype=np.int32)
        nct = np.array([ctrl.shape[2], ctrl.shape[1], ctrl.shape[0]], dtype=np.int32)
        kn = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.float64) for t in net["knots"]]))
        rc = lib.ka_host_geometry_eval(2, None, _p(deg, ctypes.c_int), _p(nct, ctypes.c_int), _p(kn), _p(ctrl), n,
                                       _p(xh), _p(x), _p(J), _p(W), None)
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


# ---- C^0 lines (paper Sec. 4.1) -------------------------------------------------------------

def _net_args(net):
    deg = np.array(net["degree"], dtype=np.int32)
    ctrl = np.asarray(net["ctrl"])
    nct = np.array([ctrl.shape[2], ctrl.shape[1], ctrl.shape[0]], dtype=np.int32)
    kn = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.float64) for t in net["knots"]]))
    return deg, nct, kn


@pytest.mark.parametrize("which", ["half_cylinder", "kinked", "blob", "annulus"])
def test_c0_lines_match_oracle(lib, which):
    from workloads import half_cylinder_net, kinked_box_net
    net = {"half_cylinder": half_cylinder_net(), "kinked": kinked_box_net(0.25, 0.6), "blob": nurbs_blob_net(3),
           "annulus": nurbs_annulus_net()}[which]
    deg, nct, kn = _net_args(net)
    nv = geometry.NurbsVolume(net["degree"], net["knots"], net["ctrl"])
    for k in range(3):
        out = np.zeros(16)
        n = lib.ka_host_c0_lines(_p(deg, ctypes.c_int), _p(nct, ctypes.c_int), _p(kn), k, _p(out), 16)
        assert tuple(out[:n]) == nv.c0_lines(k)


@pytest.mark.parametrize("seed", range(6))
def test_analysis_knots_match_oracle(lib, seed):
    from oracle import splines
    rng = np.random.default_rng(seed)
    p, nel = int(rng.integers(1, 5)), int(rng.integers(1, 9))
    mult = int(rng.integers(1, p + 2))
    lines = sorted({float(rng.integers(1, 8)) / 8 if rng.random() < 0.5 else float(rng.random()) for _ in range(2)})
    lines = np.array([l for l in lines if 0 < l < 1])
    lm = int(rng.choice([p, p + 1]))
    ref = splines.open_knots(p, nel, mult, lines=tuple(lines), line_mult=lm)
    out = np.zeros(512)
    n = lib.ka_host_analysis_knots(p, nel, mult, _p(np.ascontiguousarray(lines)), len(lines), lm, _p(out), 512)
    assert n == len(ref)
    assert np.abs(out[:n] - ref).max() < 1e-15


@pytest.mark.parametrize("p,c", [(1, 0.5), (2, 0.5), (3, 0.1), (4, 0.7)])
def test_one_sided_rows_match_oracle(lib, p, c):
    from oracle import splines
    t = splines.open_knots(p, 5, 1, lines=(c,), line_mult=p + 1)
    rng = np.random.default_rng(p)
    x = np.concatenate([np.unique(t), rng.random(20)])
    left = (rng.random(len(x)) < 0.5).astype(np.int8)
    n = splines.num_basis(t, p)
    out = np.zeros((len(x), n))
    gl = np.zeros(n, dtype=np.int8)
    lib.ka_host_bspline_rows(_p(t), len(t), p, _p(x), len(x), _p(left, ctypes.c_char), _p(out),
                             _p(gl, ctypes.c_char))
    assert np.abs(out - splines.basis_matrix(t, p, x, left=left.astype(bool))).max() < 1e-14
    assert np.array_equal(gl.astype(bool), splines.greville_left(t, p))


def test_one_sided_jacobian(lib):
    from workloads import kinked_box_net
    net = kinked_box_net(0.5, 0.3)
    xh = np.array([[0.5, 0.2, 0.7], [0.5, 0.2, 0.7], [0.3, 0.5, 0.5]])
    left = np.array([[1, 0, 0], [0, 0, 0], [1, 1, 1]], dtype=np.int8)
    deg, nct, kn = _net_args(net)
    ctrl = np.ascontiguousarray(net["ctrl"], dtype=np.float64)
    x, J, W = np.zeros((3, 3)), np.zeros(3), np.zeros(3)
    rc = lib.ka_host_geometry_eval(2, None, _p(deg, ctypes.c_int), _p(nct, ctypes.c_int), _p(kn), _p(ctrl), 3,
                                   _p(xh), _p(x), _p(J), _p(W), _p(left, ctypes.c_char))
    assert rc == 0
    nv = geometry.NurbsVolume(net["degree"], net["knots"], net["ctrl"])
    assert np.abs(J - nv.detJ(xh, left.astype(bool))).max() < 1e-14
    assert abs(J[0] - 0.6) < 1e-14 and abs(J[1] - 1.4) < 1e-14
