"""Univariate B-spline machinery (paper Sec. 3.1: tensor-product B-splines of
uniform degree p; Sec. 3.2: collocation at Greville abscissae).

Everything here is FP64 and written for clarity, not speed.
"""
import numpy as np


def open_knots(p, nel, mult=1, a=0.0, b=1.0, lines=(), line_mult=None):
    """Open knot vector on [a, b]: `nel` uniform elements plus extra lines.

    End knots are repeated p+1 times; every interior breakpoint is repeated
    `mult` times, giving C^{p-mult} continuity there (mult=1: C^{p-1}, the
    smooth solution space; mult=p: C^0, the interpolation space used for the
    rough exponential kernel, Sec. 4.1; mult=p+1: C^-1, a broken space).

    `lines` are further breakpoints, the parametric positions where the
    geometry is only C^0 (Sec. 4.1); each is repeated `line_mult` times
    (default p, C^0) instead, and added to the mesh when it is not one of the
    uniform breakpoints already.
    """
    if line_mult is None:
        line_mult = p
    if not (1 <= mult <= p + 1) or not (1 <= line_mult <= p + 1):
        raise ValueError("interior multiplicity must lie in [1, p+1]")
    inner = {}
    for k in range(1, nel):
        inner[a + (b - a) * k / nel] = mult
    for x in lines:
        x = float(x)
        if not (a < x < b):
            raise ValueError("a line must lie inside the interval")
        near = [y for y in inner if abs(y - x) <= 1e-12 * (b - a)]
        for y in near:
            del inner[y]
        inner[x] = line_mult
    knots = [a] * (p + 1)
    for x in sorted(inner):
        knots += [x] * inner[x]
    return np.array(knots + [b] * (p + 1), dtype=np.float64)


def num_basis(knots, p):
    return len(knots) - p - 1


def basis_matrix(knots, p, x, left=None):
    """All B-splines of degree p on `knots` evaluated at points x.

    Returns an array (len(x), n) built with the Cox-de Boor recursion
    B_{i,0} = 1 on [t_i, t_{i+1}),  B_{i,k} = w1 B_{i,k-1} + w2 B_{i+1,k-1},
    with 0/0 := 0.  The right end point b belongs to the last non-empty span.

    `left` (boolean per point, optional) asks for the limit from the left
    instead: B_{i,0} = 1 on (t_i, t_{i+1}].  Where the space is discontinuous
    (a knot of multiplicity p+1) the two limits differ; elsewhere they agree.
    The left end point a has no left limit and keeps the first span.
    """
    t = np.asarray(knots, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    lm = np.zeros(len(x), dtype=bool) if left is None else np.broadcast_to(np.asarray(left, dtype=bool), x.shape)
    m = len(t) - 1
    B = np.zeros((len(x), m))
    spans = [i for i in range(m) if t[i + 1] > t[i]]
    for i in spans:
        B[:, i] = np.where(lm, (t[i] < x) & (x <= t[i + 1]), (t[i] <= x) & (x < t[i + 1]))
    B[(x == t[-1]) & ~lm, spans[-1]] = 1.0
    B[(x == t[0]) & lm, spans[0]] = 1.0
    for k in range(1, p + 1):
        Bn = np.zeros((len(x), m - k))
        for i in range(m - k):
            d1 = t[i + k] - t[i]
            d2 = t[i + k + 1] - t[i + 1]
            if d1 > 0:
                Bn[:, i] += (x - t[i]) / d1 * B[:, i]
            if d2 > 0:
                Bn[:, i] += (t[i + k + 1] - x) / d2 * B[:, i + 1]
        B = Bn
    return B


def basis_derivative_matrix(knots, p, x, left=None):
    """First derivatives of all degree-p B-splines at x, shape (len(x), n):
    B'_{i,p} = p B_{i,p-1} / (t_{i+p} - t_i) - p B_{i+1,p-1} / (t_{i+p+1} - t_{i+1})
    (terms with a zero denominator dropped)."""
    t = np.asarray(knots, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = num_basis(t, p)
    Bl = basis_matrix(t, p - 1, x, left)    # degree p-1: n + 1 functions
    D = np.zeros((len(x), n))
    for i in range(n):
        d1 = t[i + p] - t[i]
        d2 = t[i + p + 1] - t[i + 1]
        if d1 > 0:
            D[:, i] += p * Bl[:, i] / d1
        if d2 > 0:
            D[:, i] -= p * Bl[:, i + 1] / d2
    return D


def greville(knots, p):
    """Greville abscissae gamma_i = (t_{i+1} + ... + t_{i+p}) / p; when the p
    knots are equal the abscissa is that knot, exactly (a rounded mean could
    land beside it)."""
    t = np.asarray(knots, dtype=np.float64)
    n = num_basis(t, p)
    return np.array([t[i + 1] if t[i + 1] == t[i + p] else t[i + 1:i + p + 1].mean() for i in range(n)])


def greville_left(knots, p):
    """Which Greville abscissae are taken as limits from the left: those that
    coincide with the right end of their own function's support inside the
    interval.  That happens only at a knot of multiplicity p+1 (C^-1), where
    the last function of the left piece and the first of the right piece
    share one abscissa; evaluating each from its own side keeps the
    interpolation matrix non-singular."""
    t = np.asarray(knots, dtype=np.float64)
    g = greville(t, p)
    return np.array([g[i] == t[i + p + 1] and t[i + p + 1] < t[-1] for i in range(len(g))], dtype=bool)


def gauss_legendre(q, a=-1.0, b=1.0):
    """q-point Gauss-Legendre rule on [a, b] (numpy's leggauss, rescaled)."""
    x, w = np.polynomial.legendre.leggauss(q)
    return a + (b - a) * (x + 1) / 2, w * (b - a) / 2


def breakpoints(knots):
    return np.unique(np.asarray(knots, dtype=np.float64))


def element_quadrature(knots, q):
    """Tensor of a q-point Gauss rule over every element (non-empty span).

    Points are ordered element by element, left to right, and within an
    element in increasing order, so the flat index is e*q + g.
    """
    br = breakpoints(knots)
    xs, ws = [], []
    for e in range(len(br) - 1):
        x, w = gauss_legendre(q, br[e], br[e + 1])
        xs.append(x)
        ws.append(w)
    return np.concatenate(xs), np.concatenate(ws)


def mass_matrix(knots_a, pa, knots_b, pb, q=None):
    """Z[i, j] = integral of B^a_i B^b_j over the parameter interval.

    Both spaces must share the breakpoints.  A Gauss rule with
    q = ceil((pa+pb+1)/2) points per element integrates the product exactly.
    """
    if not np.array_equal(breakpoints(knots_a), breakpoints(knots_b)):
        raise ValueError("spaces must share the mesh")
    if q is None:
        q = (pa + pb) // 2 + 1
    x, w = element_quadrature(knots_a, q)
    Ba = basis_matrix(knots_a, pa, x)
    Bb = basis_matrix(knots_b, pb, x)
    return (Ba * w[:, None]).T @ Bb


def collocation_matrix(knots, p, pts):
    """B[a, c] = B_c(pts_a): rows are points, columns are basis functions."""
    return basis_matrix(knots, p, pts)
