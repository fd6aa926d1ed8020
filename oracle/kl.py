"""Truncated Karhunen-Loeve expansion of the random field (paper Sec. 2,
eq. kle), evaluated on a tensor grid of parametric points:

    alpha_M(x, s) = mu + sum_{i=1..M} sqrt(lambda_i) phi_i(x) xi_i(s),

with phi_i the computed eigenfunctions normalised in L^2(D) (the expansion
assumes orthonormal eigenfunctions) and xi_i(s) the draws of sample s, passed
in.  Test infrastructure: plain FP64 numpy.

The eigenfunction with coefficient vector v lives in the method's trial space:
  * Galerkin (IBQ and standard, Sec. 3.1): phi(x) = sum_j v_j B_j(xh) / sqrt|det DF(xh)|
    for x = F(xh), so that int_D phi^2 dx = v^T Z v;
  * collocation (Sec. 3.2): phi(x) = sum_j v_j R_j(xh), R_j the NURBS trial functions
    (tensor weights), or B_j(xh) / W(xh) on a general NURBS volume.
The L^2(D) norm int_D phi^2 dx = int phi(F(xh))^2 |det DF(xh)| dxh is taken
with a Gauss rule per element and direction: p + 1 points for Galerkin (exact:
the integrand is (sum_j v_j B_j)^2), the collocation rule's nq points for
collocation.
"""
import numpy as np

from . import kron, splines
from .collocation import Collocation, nurbs_basis_1d


def _is_collocation(disc):
    return isinstance(disc, Collocation)


def _trial_1d(disc, k, x):
    """Univariate factor of the trial space in direction k, rows are points."""
    t = disc.knots[k]
    if _is_collocation(disc) and not disc.rational:
        return nurbs_basis_1d(t, disc.p, lambda s: disc.domain.weight1d(k, s), np.asarray(x))
    return splines.basis_matrix(t, disc.p, np.asarray(x))


def grid_points(grid):
    """Tensor grid of parametric points, index i1 + n1 (i2 + n2 i3)."""
    g3, g2, g1 = np.meshgrid(grid[2], grid[1], grid[0], indexing="ij")
    return np.stack([g1.ravel(), g2.ravel(), g3.ravel()], axis=-1)


def _point_scale(disc, xh):
    if _is_collocation(disc):
        return 1.0 / disc.domain.weight(xh) if disc.rational else np.ones(len(xh))
    return 1.0 / np.sqrt(np.abs(disc.domain.detJ(xh)))


def eigenfunctions(disc, V, grid):
    """phi_i at the grid points: (P, M) for V of shape (N, M)."""
    E = [_trial_1d(disc, k, grid[k]) for k in range(3)]
    Phi = kron.kron_apply(E, np.asarray(V, dtype=np.float64))
    return _point_scale(disc, grid_points(grid))[:, None] * Phi


def l2_norms(disc, V):
    """||phi_i||_{L^2(D)} by the Gauss rule described in the module docstring."""
    q = disc.nq if _is_collocation(disc) else disc.p + 1
    rules = [splines.element_quadrature(t, q) for t in disc.knots]
    grid = [r[0] for r in rules]
    w3, w2, w1 = np.meshgrid(rules[2][1], rules[1][1], rules[0][1], indexing="ij")
    w = (w1 * w2 * w3).ravel() * np.abs(disc.domain.detJ(grid_points(grid)))
    Phi = eigenfunctions(disc, V, grid)
    return np.sqrt(w @ Phi ** 2)


def sample(disc, lam, V, grid, xi, mu=0.0):
    """Fields at the grid points, shape (P, S), for draws xi of shape (M, S)."""
    lam = np.asarray(lam, dtype=np.float64)
    Phi = eigenfunctions(disc, V, grid)
    scale = np.sqrt(lam) / l2_norms(disc, V)
    return mu + Phi @ (scale[:, None] * np.asarray(xi, dtype=np.float64))
