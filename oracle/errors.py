"""Eigenvalue error measures (paper Sec. 4.1: relative error eps_i of the i-th
eigenvalue against a reference and its mean over the first M)."""
import numpy as np


def rel_errors(lam_ref, lam):
    """eps_i = |lam_ref_i - lam_i| / lam_ref_i."""
    lam_ref = np.asarray(lam_ref, dtype=np.float64)
    return np.abs(lam_ref - np.real(lam)) / np.abs(lam_ref)


def mean_rel_error(lam_ref, lam):
    """mean of eps_i over the given eigenvalues."""
    return float(np.mean(rel_errors(lam_ref, lam)))


def floored_rel_errors(lam_ref, lam, tau=1e-2):
    """|lam_ref_i - lam_i| / max(lam_ref_i, tau * lam_ref_1).

    Reading for single-precision arithmetic: an FP32 operator carries an
    absolute error of order eps32 * lambda_1, so relative errors of small
    eigenvalues are measured against the floor tau * lambda_1."""
    lam_ref = np.asarray(lam_ref, dtype=np.float64)
    den = np.maximum(np.abs(lam_ref), tau * np.abs(lam_ref[0]))
    return np.abs(lam_ref - np.real(lam)) / den


def clusters(lam_ref, rtol=1e-8):
    """Group indices of (sorted, descending) eigenvalues whose relative gap
    is below rtol: degenerate clusters of the reference spectrum."""
    lam_ref = np.asarray(lam_ref)
    groups, cur = [], [0]
    for i in range(1, len(lam_ref)):
        if abs(lam_ref[i] - lam_ref[i - 1]) <= rtol * abs(lam_ref[i - 1]):
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    groups.append(cur)
    return groups


def subspace_angle(U, V, G=None):
    """Largest principal angle between span(U) and span(V) in the inner
    product <x, y> = x^T G y (G = identity if None)."""
    import scipy.linalg as sla
    if G is None:
        G = np.eye(U.shape[0])
    def orth(X):
        R = sla.cholesky(X.T @ G @ X)
        return X @ np.linalg.inv(R)
    Qu, Qv = orth(U), orth(V)
    s = np.linalg.svd(Qu.T @ G @ Qv, compute_uv=False)
    return float(np.arccos(np.clip(s.min(), -1.0, 1.0)))
