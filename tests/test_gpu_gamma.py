"""Parity of the fused kernel product (ka_gamma_apply) with the FP64 oracle.

Bar: |Z - Z_ref| <= tol * (|Gamma| |Y|) elementwise, the natural scale of a
sum of products.  FP32 tiles + FP32 MFMA: the coordinate prescale and the
difference give ~4e-7 relative error in Gamma, exp2 ~1e-7, and FP32
accumulation over ~400 MFMA steps ~sqrt(400) u = 1.2e-6 typical, so
tol = 1e-5 (~170 u) leaves headroom for the worst case.  Split BF16x3: the
dropped lo*lo product and the BF16 rounding of the lo parts cost up to
2^-16 = 1.5e-5 per product on top, so tol = 6e-5.  Row blocks of small
extent take the centred Gram form of the Gaussian exponent, whose terms are
of size R^2 <= 20 (scaled units) instead of |x - y|^2: a few units of 2^-24
R^2 in the exponent, at most ~4e-6 relative in Gamma, inside the same bars.
"""
import numpy as np
import pytest
import torch

import paper_2101_00629_amd as K
from oracle import kernels
from workloads import normal_block, tensor_grid_points, uniform_points

pytestmark = pytest.mark.gpu

TOL = {K.KA_FP32: 1e-5, K.KA_BF16X3: 6e-5}
KNAME = {K.KA_GAUSSIAN: "gaussian", K.KA_EXP_L1: "exponential"}


def _run(kernel, sigma, ell, Xr, Xc, Y, precision):
    dev = "cuda"
    xr = torch.tensor(Xr, dtype=torch.float32, device=dev)
    xc = torch.tensor(Xc, dtype=torch.float32, device=dev)
    y = torch.tensor(Y, dtype=torch.float32, device=dev)
    z = torch.full((Xr.shape[0], Y.shape[1]), float("nan"), dtype=torch.float32, device=dev)
    nbytes = K.ka_gamma_workspace(Xr.shape[0], Xc.shape[0], Y.shape[1], precision)
    work = torch.empty(max(nbytes // 4, 1), dtype=torch.float32, device=dev)
    K.ka_gamma_apply(kernel, sigma, ell, xr, xc, y, z, precision, work)
    torch.cuda.synchronize()
    return z.cpu().numpy().astype(np.float64)


def _reference(kernel, sigma, ell, Xr, Xc, Y):
    # the oracle sees the same FP32-rounded inputs the device sees
    Xr = Xr.astype(np.float32).astype(np.float64)
    Xc = Xc.astype(np.float32).astype(np.float64)
    Y = Y.astype(np.float32).astype(np.float64)
    G = kernels.kernel_matrix(KNAME[kernel], Xr, Xc, ell, sigma)
    return G @ Y, np.abs(G) @ np.abs(Y)


@pytest.mark.parametrize("precision", [K.KA_FP32, K.KA_BF16X3])
@pytest.mark.parametrize("kernel,ell", [(K.KA_GAUSSIAN, 0.3), (K.KA_EXP_L1, 0.5)])
@pytest.mark.parametrize("b", [16, 32, 64])
def test_gamma_matches_oracle_ragged(precision, kernel, ell, b):
    nr, nc = 1000, 1531           # several row blocks and column tiles, ragged tails
    Xr = uniform_points(1, nr)
    Xc = uniform_points(2, nc, lo=(-0.2, 0, 0), hi=(1.0, 1.3, 0.9))
    Y = normal_block(3, nc, b)
    Z = _run(kernel, 1.3, ell, Xr, Xc, Y, precision)
    ref, scale = _reference(kernel, 1.3, ell, Xr, Xc, Y)
    err = np.abs(Z - ref) / scale
    assert np.isfinite(Z).all()
    assert err.max() < TOL[precision], err.max()


@pytest.mark.parametrize("precision", [K.KA_FP32, K.KA_BF16X3])
@pytest.mark.parametrize("nr,nc", [(200, 20011), (600, 50000)])
def test_gamma_split_k_path(precision, nr, nc):
    # few rows, many columns: the column range is split over workgroups (16
    # and 24 splits: the XCD-grouped grid, with one and three row blocks)
    b = 16
    assert K.ka_gamma_workspace(nr, nc, b, precision) > 0
    Xr = uniform_points(4, nr)
    Xc = uniform_points(5, nc)
    Y = normal_block(6, nc, b)
    Z = _run(K.KA_GAUSSIAN, 1.0, 0.5, Xr, Xc, Y, precision)
    ref, scale = _reference(K.KA_GAUSSIAN, 1.0, 0.5, Xr, Xc, Y)
    assert (np.abs(Z - ref) / scale).max() < TOL[precision]


def _block_r2(X, ell, rows):
    """Half-diagonal^2 of each row block's box in the kernel's scaled
    coordinates (sqrt(log2 e) / ell): blocks at or below 20 take the centred
    Gram form of the Gaussian product, wider ones the difference form."""
    Xs = X.astype(np.float32).astype(np.float64) * (np.sqrt(np.log2(np.e)) / ell)
    out = []
    for i in range(0, len(Xs), rows):
        B = Xs[i:i + rows]
        out.append((((B.max(0) - B.min(0)) / 2) ** 2).sum())
    return np.array(out)


@pytest.mark.parametrize("precision", [K.KA_FP32, K.KA_BF16X3])
@pytest.mark.parametrize("b", [16, 32, 64])
def test_gamma_gram_and_difference_forms_in_one_launch(precision, b):
    # rows: a 13 x 11 x 9 tensor grid in its natural order (compact row
    # blocks: centred Gram form), then a random cloud in [-1, 2]^3 (wide
    # blocks: difference form); ragged row and column counts
    ell = 0.3
    grid = tensor_grid_points((13, 11, 9))
    Xr = np.concatenate([grid, uniform_points(21, 700, lo=(-1, -1, -1), hi=(2, 2, 2))])
    Xc = np.concatenate([tensor_grid_points((17, 13, 7), "quarter_annulus") * 0.6, uniform_points(22, 300)])
    rows = 128 if b == 64 else 256            # rows per workgroup of the kernel product
    r2 = _block_r2(Xr, ell, rows)
    ngrid = len(grid) // rows                  # blocks made of grid rows only
    assert (r2[:ngrid] <= 20).all() and (r2[ngrid + 1:] > 20).all()
    Y = normal_block(23, len(Xc), b)
    Z = _run(K.KA_GAUSSIAN, 1.1, ell, Xr, Xc, Y, precision)
    ref, scale = _reference(K.KA_GAUSSIAN, 1.1, ell, Xr, Xc, Y)
    assert np.isfinite(Z).all()
    err = np.abs(Z - ref) / scale
    assert err.max() < TOL[precision], err.max()


@pytest.mark.parametrize("precision", [K.KA_FP32, K.KA_BF16X3])
def test_gamma_gram_form_split_k(precision):
    # grid rows (Gram form) against many columns: split-K partial sums of the
    # Gram form, each scaled by the rows' factor before the reduction
    nr_grid, nc, b, ell = (10, 10, 2), 20011, 16, 0.4
    Xr = tensor_grid_points(nr_grid)
    assert (_block_r2(Xr, ell, 256) <= 20).all()
    Xc = uniform_points(24, nc)
    Y = normal_block(25, nc, b)
    assert K.ka_gamma_workspace(len(Xr), nc, b, precision) > 0
    Z = _run(K.KA_GAUSSIAN, 1.0, ell, Xr, Xc, Y, precision)
    ref, scale = _reference(K.KA_GAUSSIAN, 1.0, ell, Xr, Xc, Y)
    assert (np.abs(Z - ref) / scale).max() < TOL[precision]


def test_gamma_constant_kernel_exact_sum():
    # ell = inf: Gamma == 1 exactly (exp2(0)), Z = sigma^2 * column sums of Y
    nr, nc, b = 77, 300, 16
    Y = np.round(normal_block(7, nc, b) * 64) / 64       # exactly representable, exact sums
    Z = _run(K.KA_GAUSSIAN, 1.0, np.inf, uniform_points(8, nr), uniform_points(9, nc), Y, K.KA_FP32)
    assert np.array_equal(Z, np.tile(Y.sum(axis=0), (nr, 1)))


def test_gamma_edge_sizes():
    for nr, nc in ((1, 1), (1, 700), (333, 1), (65, 64)):
        Xr, Xc = uniform_points(10, nr), uniform_points(11, nc)
        Y = normal_block(12, nc, 32)
        Z = _run(K.KA_EXP_L1, 0.7, 0.4, Xr, Xc, Y, K.KA_FP32)
        ref, scale = _reference(K.KA_EXP_L1, 0.7, 0.4, Xr, Xc, Y)
        assert (np.abs(Z - ref) / scale).max() < TOL[K.KA_FP32], (nr, nc)
    # no columns: Z = 0
    Z = _run(K.KA_GAUSSIAN, 1.0, 0.5, uniform_points(13, 50), np.zeros((0, 3)), np.zeros((0, 16)), K.KA_FP32)
    assert np.array_equal(Z, np.zeros((50, 16)))


def test_gamma_rejects_bad_arguments():
    x = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    y = torch.zeros((4, 16), dtype=torch.float32, device="cuda")
    z = torch.zeros((4, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(K.KAError):
        K.ka_gamma_apply(K.KA_GAUSSIAN, 1.0, -1.0, x, x, y, z)
    y24 = torch.zeros((4, 24), dtype=torch.float32, device="cuda")
    with pytest.raises(K.KAError):
        K.ka_gamma_apply(K.KA_GAUSSIAN, 1.0, 1.0, x, x, y24, y24)
