"""Geometry maps F : [0,1]^3 -> D and |det DF| (paper Sec. 3.1, the map F
from the reference to the physical domain; Sec. 3.2, NURBS geometry).

Three kinds of domain are used by the workloads:

* Box [lo, hi]: F(xh) = lo + (hi - lo) * xh, |det DF| = prod(hi - lo).
* Quarter annulus r in [r0, r1], angle in [0, pi/2], extruded to `height`:
  F(xi, eta, zeta) = ((r0 + (r1 - r0) eta) C(xi), height zeta), where C is the
  exact rational quadratic quarter circle with control points (1,0), (1,1),
  (0,1) and weights 1, 1/sqrt(2), 1.  Since C is a unit vector and C' is
  orthogonal to it, |det DF| = (r1 - r0) * r(eta) * |C'(xi)| * height.
* A general single-patch NURBS volume, given by its control net (NurbsVolume).
"""
import numpy as np

W_MID = 1.0 / np.sqrt(2.0)


class Box:
    kind = "box"

    def __init__(self, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)

    def map(self, xh, left=None):
        xh = np.asarray(xh, dtype=np.float64)
        return self.lo + (self.hi - self.lo) * xh

    def detJ(self, xh, left=None):
        xh = np.asarray(xh, dtype=np.float64)
        return np.full(xh.shape[:-1], np.prod(self.hi - self.lo))

    def c0_lines(self, k):
        """Interior parametric positions where the map is only C^0 (none)."""
        return ()

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

    def map(self, xh, left=None):
        xh = np.asarray(xh, dtype=np.float64)
        C, _ = quarter_circle(xh[..., 0])
        r = self.r0 + (self.r1 - self.r0) * xh[..., 1]
        return np.stack([r * C[..., 0], r * C[..., 1], self.height * xh[..., 2]], axis=-1)

    def detJ(self, xh, left=None):
        xh = np.asarray(xh, dtype=np.float64)
        _, dC = quarter_circle(xh[..., 0])
        r = self.r0 + (self.r1 - self.r0) * xh[..., 1]
        return (self.r1 - self.r0) * r * np.hypot(dC[..., 0], dC[..., 1]) * self.height

    def volume(self):
        return np.pi / 4 * (self.r1 ** 2 - self.r0 ** 2) * self.height

    def c0_lines(self, k):
        return ()

    def weight1d(self, k, t):
        """NURBS weight function of direction k: D(xi) along xi, 1 otherwise."""
        if k == 0:
            return circle_weight(t)
        return np.ones(np.shape(t))


class NurbsVolume:
    """Single-patch NURBS volume (paper Sec. 3.2: NURBS geometry):
    F(xh) = sum_j w_j P_j N_j(xh) / W(xh),  W(xh) = sum_j w_j N_j(xh),
    N_j the tensor-product B-splines of the given degrees and knot vectors.
    ctrl has shape (n3, n2, n1, 4) with rows (x, y, z, w).

    The collocation trial space on such a volume is spanned by B_j / W
    (B_j the analysis B-splines): the same space as the NURBS functions
    w_j B_j / W, so `rational` tells the collocation oracle to use it."""
    kind = "nurbs"
    rational = True

    def __init__(self, degree, knots, ctrl):
        self.p = tuple(int(d) for d in degree)
        self.t = [np.asarray(k, dtype=np.float64) for k in knots]
        ctrl = np.asarray(ctrl, dtype=np.float64)
        self.ctrl = ctrl
        # homogeneous control points (w x, w y, w z, w)
        self.H = np.concatenate([ctrl[..., :3] * ctrl[..., 3:4], ctrl[..., 3:4]], axis=-1)

    def c0_lines(self, k):
        """Interior knots of direction k repeated at least p_k times: there the
        map is only C^0 (Sec. 4.1), e.g. where two patches meet."""
        t, p = self.t[k], self.p[k]
        vals, counts = np.unique(t, return_counts=True)
        return tuple(float(v) for v, c in zip(vals, counts) if t[0] < v < t[-1] and c >= p)

    def _sums(self, xh, left=None):
        """Homogeneous sum and its three parametric derivatives at points xh (m, 3);
        left (m, 3) booleans take direction k's limit from the left."""
        from . import splines
        lf = [None if left is None else left[:, k] for k in range(3)]
        B = [splines.basis_matrix(self.t[k], self.p[k], xh[:, k], lf[k]) for k in range(3)]
        D = [splines.basis_derivative_matrix(self.t[k], self.p[k], xh[:, k], lf[k]) for k in range(3)]
        S = np.einsum("ma,mb,mc,cbad->md", B[0], B[1], B[2], self.H)
        S1 = np.einsum("ma,mb,mc,cbad->md", D[0], B[1], B[2], self.H)
        S2 = np.einsum("ma,mb,mc,cbad->md", B[0], D[1], B[2], self.H)
        S3 = np.einsum("ma,mb,mc,cbad->md", B[0], B[1], D[2], self.H)
        return S, (S1, S2, S3)

    def _eval(self, xh, left=None, chunk=4096):
        xh = np.asarray(xh, dtype=np.float64)
        shape = xh.shape[:-1]
        flat = xh.reshape(-1, 3)
        lflat = None if left is None else np.broadcast_to(np.asarray(left, dtype=bool), xh.shape).reshape(-1, 3)
        X = np.empty((len(flat), 3))
        J = np.empty(len(flat))
        W = np.empty(len(flat))
        for s0 in range(0, len(flat), chunk):
            S, dS = self._sums(flat[s0:s0 + chunk], None if lflat is None else lflat[s0:s0 + chunk])
            w = S[:, 3]
            x = S[:, :3] / w[:, None]
            # dF[:, c, k] = (dS_k[c] - x_c dS_k[w]) / w
            dF = np.stack([(d[:, :3] - x * d[:, 3:4]) / w[:, None] for d in dS], axis=-1)
            X[s0:s0 + chunk] = x
            J[s0:s0 + chunk] = np.linalg.det(dF)
            W[s0:s0 + chunk] = w
        return X.reshape(shape + (3,)), J.reshape(shape), W.reshape(shape)

    def map(self, xh, left=None):
        return self._eval(xh, left)[0]

    def detJ(self, xh, left=None):
        """|det DF|; at a C^0 line it jumps, and `left` picks the side."""
        return np.abs(self._eval(xh, left)[1])

    def weight(self, xh, left=None):
        """The weight function W at parametric points."""
        return self._eval(xh, left)[2]

    def volume(self, q=None):
        """Integral of |det DF| by Gauss-Legendre on every knot span (q per span and direction)."""
        from . import splines
        rules = []
        for k in range(3):
            x, w = splines.element_quadrature(self.t[k], q or (2 * self.p[k] + 6))
            rules.append((x, w))
        g3, g2, g1 = np.meshgrid(rules[2][0], rules[1][0], rules[0][0], indexing="ij")
        w3, w2, w1 = np.meshgrid(rules[2][1], rules[1][1], rules[0][1], indexing="ij")
        xh = np.stack([g1.ravel(), g2.ravel(), g3.ravel()], axis=-1)
        return float(np.sum(self.detJ(xh) * (w1 * w2 * w3).ravel()))


def c0_lines(domain, k):
    """The domain's C^0 lines in parametric direction k (none for closed-form maps)."""
    f = getattr(domain, "c0_lines", None)
    return tuple(f(k)) if f else ()


def make_domain(name, **kw):
    if name in ("cube", "box"):
        return Box(kw.get("lo", (0.0, 0.0, 0.0)), kw.get("hi", (1.0, 1.0, 1.0)))
    if name in ("quarter_annulus", "annulus"):
        return QuarterAnnulus(kw.get("r0", 1.0), kw.get("r1", 2.0), kw.get("height", 1.0))
    if name == "nurbs":
        n = kw["nurbs"]
        return NurbsVolume(n["degree"], n["knots"], n["ctrl"])
    raise ValueError(name)
