"""Covariance kernels Gamma(x, x') (paper Sec. 2, covariance function; Sec. 4.1
exponential kernel, Sec. 4.2 Gaussian kernel).

The paper does not print the formulas.  Read as:
  gaussian     sigma^2 exp(-|x - x'|_2^2 / ell^2)
  exponential  sigma^2 exp(-|x - x'|_1 / ell)
Both are separable across coordinates, which the product-of-1D oracle uses.
"""
import numpy as np

GAUSSIAN = "gaussian"
EXPONENTIAL = "exponential"


def kernel_matrix(kind, X, Y, ell, sigma=1.0):
    """Dense Gamma[a, c] = Gamma(X[a], Y[c]) in FP64; X (n,d), Y (m,d)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    if Y.ndim == 1:
        Y = Y[:, None]
    diff = X[:, None, :] - Y[None, :, :]
    if kind == GAUSSIAN:
        if np.isinf(ell):
            return np.full((len(X), len(Y)), sigma ** 2)
        return sigma ** 2 * np.exp(-np.sum(diff ** 2, axis=-1) / ell ** 2)
    if kind == EXPONENTIAL:
        return sigma ** 2 * np.exp(-np.sum(np.abs(diff), axis=-1) / ell)
    raise ValueError(kind)


def kernel_1d_factor(kind, x, y, ell):
    """One coordinate's factor of a separable kernel (sigma = 1)."""
    return kernel_matrix(kind, np.asarray(x)[:, None], np.asarray(y)[:, None], ell, 1.0)
