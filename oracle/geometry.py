"""Geometry maps F : [0,1]^3 -> D and |det DF| (paper Sec. 3.1, the map F
from the reference to the physical domain; Sec. 3.2, NURBS geometry).

Two domains are used by the workloads:

* Box [lo, hi]: F(xh) = lo + (hi - lo) * xh, |det DF| = prod(hi - lo).
* Quarter annulus r in [r0, r1], angle in [0, pi/2], extruded to `height`:
  F(xi, eta, zeta) = ((r0 + (r1 - r0) eta) C(xi), height zeta), where C is the
  exact rational quadratic quarter circle with control points (1,0), (1,1),
  (0,1) and weights 1, 1/sqrt(2), 1.  Since C is a unit vector and C' is
  orthogonal to it, |det DF| = (r1 - r0) * r(eta) * |C'(xi)| * height.
"""
import numpy as np

W_MID = 1.0 / np.sqrt(2.0)


class Box:
    kind = "box"

    def __init__(self, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)

    def map(self, xh):
        xh = np.asarray(xh, dtype=np.float64)
        return self.lo + (self.hi - self.lo) * xh

    def detJ(self, xh):
        xh = np.asarray(xh, dtype=np.float64)
        return np.full(xh.shape[:-1], np.prod(self.hi - self.lo))

    def volume(self):
        return float(np.prod(self.hi - self.lo))

    # separable factors, one per parametric direction
    def map1d(self, k, t):
        return self.lo[k] + (self.hi[k] - self.lo[k]) * np.asarray(t)

    def detJ1d(self, k, t):
        return np.full(np.shape(t), self.hi[k] - self.lo[k])

    def weight1d(self, k, t):
        """NURBS weight function of direction k (1: plain B-splines)."""
        return np.ones(np.shape(t))


def quarter_circle(xi):
    """Rational quadratic quarter circle C(xi) and its derivative C'(xi)."""
    xi = np.asarray(xi, dtype=np.float64)
    b0, b1, b2 = (1 - xi) ** 2, 2 * xi * (1 - xi), xi ** 2
    db0, db1, db2 = -2 * (1 - xi), 2 - 4 * xi, 2 * xi
    D = b0 + W_MID * b1 + b2
    dD = db0 + W_MID * db1 + db2
    Nx = b0 + W_MID * b1
    Ny = W_MID * b1 + b2
    dNx = db0 + W_MID * db1
    dNy = W_MID * db1 + db2
    C = np.stack([Nx / D, Ny / D], axis=-1)
    dC = np.stack([(dNx * D - Nx * dD) / D ** 2, (dNy * D - Ny * dD) / D ** 2], axis=-1)
    return C, dC


def circle_weight(xi):
    """Denominator D(xi) of the rational quarter circle (a quadratic)."""
    xi = np.asarray(xi, dtype=np.float64)
    return (1 - xi) ** 2 + W_MID * 2 * xi * (1 - xi) + xi ** 2


class QuarterAnnulus:
    kind = "quarter_annulus"

    def __init__(self, r0=1.0, r1=2.0, height=1.0):
        self.r0, self.r1, self.height = float(r0), float(r1), float(height)

    def map(self, xh):
        xh = np.asarray(xh, dtype=np.float64)
        C, _ = quarter_circle(xh[..., 0])
        r = self.r0 + (self.r1 - self.r0) * xh[..., 1]
        return np.stack([r * C[..., 0], r * C[..., 1], self.height * xh[..., 2]], axis=-1)

    def detJ(self, xh):
        xh = np.asarray(xh, dtype=np.float64)
        _, dC = quarter_circle(xh[..., 0])
        r = self.r0 + (self.r1 - self.r0) * xh[..., 1]
        return (self.r1 - self.r0) * r * np.hypot(dC[..., 0], dC[..., 1]) * self.height

    def volume(self):
        return np.pi / 4 * (self.r1 ** 2 - self.r0 ** 2) * self.height

    def weight1d(self, k, t):
        """NURBS weight function of direction k: D(xi) along xi, 1 otherwise."""
        if k == 0:
            return circle_weight(t)
        return np.ones(np.shape(t))


def make_domain(name, **kw):
    if name in ("cube", "box"):
        return Box(kw.get("lo", (0.0, 0.0, 0.0)), kw.get("hi", (1.0, 1.0, 1.0)))
    if name in ("quarter_annulus", "annulus"):
        return QuarterAnnulus(kw.get("r0", 1.0), kw.get("r1", 2.0), kw.get("height", 1.0))
    raise ValueError(name)
