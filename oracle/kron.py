"""Action of Kronecker-product matrices (paper Sec. 3.1: Z = Z_d x ... x Z_1,
L^-1 = L_d^-1 x ... x L_1^-1, and the Kronecker matrices M and B~).

Index convention: a 3D index (i1, i2, i3) is flattened as
i = i1 + n1 * (i2 + n2 * i3), so direction 1 runs fastest and the matrix is
A3 x A2 x A1 in numpy's np.kron order (first factor slowest).
"""
import numpy as np


def kron3(A1, A2, A3):
    """Explicit A3 (x) A2 (x) A1 (small sizes only)."""
    return np.kron(A3, np.kron(A2, A1))


def kron_apply(mats, X):
    """(A3 x A2 x A1) @ X for X of shape (n1*n2*n3, b) or (n1*n2*n3,).

    Uses the defining identity of the Kronecker product on the tensor view
    X[i3, i2, i1, :], contracting each factor with its own index.
    """
    A1, A2, A3 = mats
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    b = X.shape[1]
    T = X.reshape(A3.shape[1], A2.shape[1], A1.shape[1], b)
    T = np.einsum("ac,zycj->zyaj", A1, T)
    T = np.einsum("ac,zcxj->zaxj", A2, T)
    T = np.einsum("ac,cyxj->ayxj", A3, T)
    out = T.reshape(-1, b)
    return out[:, 0] if vec else out


def kron_solve(solvers, X):
    """Apply (A3 x A2 x A1)^-1 given per-direction solve callables."""
    s1, s2, s3 = solvers
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    b = X.shape[1]
    n1 = s1.n
    n2 = s2.n
    n3 = s3.n
    T = X.reshape(n3, n2, n1, b)
    # direction 1: fibres along the last-but-one axis
    T = np.moveaxis(s1(np.moveaxis(T, 2, 0).reshape(n1, -1)).reshape(n1, n3, n2, b), 0, 2)
    T = np.moveaxis(s2(np.moveaxis(T, 1, 0).reshape(n2, -1)).reshape(n2, n3, n1, b), 0, 1)
    T = s3(T.reshape(n3, -1)).reshape(n3, n2, n1, b)
    out = T.reshape(-1, b)
    return out[:, 0] if vec else out
