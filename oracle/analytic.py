"""Closed-form eigenpairs of the 1D exponential kernel exp(-|x - y| / ell) on
an interval of length 2a (classical result of Ghanem & Spanos, the paper's
reference for the K-L expansion of random fields).

With c = 1/ell the eigenvalues are lambda = 2c / (w^2 + c^2), where
  even modes  cos(w x) / sqrt(a + sin(2wa)/(2w)):  c - w tan(w a) = 0,
  odd modes   sin(w x) / sqrt(a - sin(2wa)/(2w)):  w + c tan(w a) = 0,
x measured from the interval centre.
"""
import numpy as np
from scipy.optimize import brentq


def exponential_1d(n, ell, length=1.0):
    """First n eigenvalues (descending) with their frequencies and parity."""
    a = length / 2.0
    c = 1.0 / ell
    out = []
    eps = 1e-12
    k = 0
    while len(out) < 2 * n + 2:
        # even root in (k pi/a, (k+1/2) pi/a)
        lo, hi = k * np.pi / a + eps, (k + 0.5) * np.pi / a - eps
        w = brentq(lambda w: c * np.cos(w * a) - w * np.sin(w * a), lo, hi)
        out.append((2 * c / (w * w + c * c), w, 0))
        # odd root in ((k+1/2) pi/a, (k+1) pi/a)
        lo, hi = (k + 0.5) * np.pi / a + eps, (k + 1) * np.pi / a - eps
        w = brentq(lambda w: w * np.cos(w * a) + c * np.sin(w * a), lo, hi)
        out.append((2 * c / (w * w + c * c), w, 1))
        k += 1
    out.sort(key=lambda t: -t[0])
    out = out[:n]
    return (np.array([o[0] for o in out]), np.array([o[1] for o in out]),
            np.array([o[2] for o in out]))


def exponential_1d_eigfun(w, parity, x, length=1.0, x0=None):
    a = length / 2.0
    x0 = a if x0 is None else x0
    s = np.asarray(x) - x0
    if parity == 0:
        return np.cos(w * s) / np.sqrt(a + np.sin(2 * w * a) / (2 * w))
    return np.sin(w * s) / np.sqrt(a - np.sin(2 * w * a) / (2 * w))


def exponential_box(M, ell, lengths=(1.0, 1.0, 1.0), sigma=1.0, n1d=60):
    """Largest M eigenvalues of sigma^2 exp(-|x-y|_1 / ell) on a box."""
    lams = [exponential_1d(n1d, ell, L)[0] for L in lengths]
    P = (lams[2][:, None, None] * lams[1][None, :, None] * lams[0][None, None, :]).ravel()
    return sigma ** 2 * np.sort(P)[::-1][:M]
