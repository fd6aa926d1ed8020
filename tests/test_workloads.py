"""CPU checks of the seeded input generators that the tests and the benchmark
share (no arithmetic of the method lives there)."""
import numpy as np

from workloads import normal_block, tensor_grid_points, uniform_points


def test_tensor_grid_cube_order_and_spacing():
    X = tensor_grid_points((3, 4, 5))
    assert X.shape == (60, 3)
    # first direction fastest, then the second, then the third
    assert np.array_equal(X[:3, 0], [0.0, 0.5, 1.0]) and np.all(X[:3, 1:] == 0.0)
    assert np.allclose(X[3], [0.0, 1.0 / 3.0, 0.0]) and np.allclose(X[12], [0.0, 0.0, 0.25])
    assert np.allclose(np.unique(X[:, 2]), np.linspace(0.0, 1.0, 5))


def test_tensor_grid_quarter_annulus_geometry():
    X = tensor_grid_points((9, 3, 2), "quarter_annulus")
    r = np.hypot(X[:, 0], X[:, 1])
    assert np.allclose(np.unique(np.round(r, 12)), [1.0, 1.5, 2.0])
    assert X[:, 0].min() >= -1e-15 and X[:, 1].min() >= -1e-15        # first quadrant
    assert np.allclose(np.unique(X[:, 2]), [0.0, 1.0])
    # the first direction runs along the arc at fixed radius and height
    assert np.allclose(r[:9], 1.0) and np.allclose(np.arctan2(X[:9, 1], X[:9, 0]), np.linspace(0, np.pi / 2, 9))


def test_seeded_draws_are_reproducible():
    assert np.array_equal(uniform_points(3, 10), uniform_points(3, 10))
    assert np.array_equal(normal_block(4, 7, 16), normal_block(4, 7, 16))
    assert not np.array_equal(uniform_points(3, 10), uniform_points(4, 10))
