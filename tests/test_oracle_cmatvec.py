"""The C OpenMP oracle product against the dense numpy kernel matrix (no GPU)."""
import numpy as np
import pytest

from oracle import cmatvec, kernels


@pytest.mark.parametrize("kind", ["gaussian", "exponential"])
def test_c_product_matches_dense_definition(kind):
    rng = np.random.default_rng(11)
    Xr, Xc = rng.random((301, 3)), 2 * rng.random((417, 3)) - 0.5
    Y = rng.standard_normal((417, 5))
    rs, cs = rng.random(301) + 0.5, rng.random(417) + 0.5
    Z = cmatvec.gamma_apply(kind, 1.4, 0.3, Xr, Xc, Y, rs=rs, cs=cs)
    ref = rs[:, None] * (kernels.kernel_matrix(kind, Xr, Xc, 0.3, 1.4) @ (cs[:, None] * Y))
    assert np.abs(Z - ref).max() < 1e-13 * np.abs(ref).max()
    z1 = cmatvec.gamma_apply(kind, 1.4, 0.3, Xr, Xc, Y[:, 0])
    assert z1.shape == (301,)
