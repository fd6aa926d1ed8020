"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: only problem descriptors
(domain, degree, mesh, kernel, ...) of the workloads and seeded random draws
(start blocks, dense blocks, point clouds, request streams).
"""
import math

import numpy as np

GAUSSIAN = "gaussian"
EXPONENTIAL = "exponential"
GALERKIN = "galerkin"
COLLOCATION = "collocation"


def problem(method, domain, p, nel, kernel, ell, sigma=1.0, M=10, block=16, precision="fp32",
            interp_mult=None, nq=None, name=None, **domain_kw):
    """Plain descriptor of one K-L problem."""
    d = dict(method=method, domain=domain, p=int(p), nel=tuple(int(e) for e in nel), kernel=kernel,
             ell=float(ell), sigma=float(sigma), M=int(M), block=int(block), precision=precision,
             interp_mult=interp_mult, nq=nq, name=name)
    d.update(domain_kw)
    return d


def small_cube(method=GALERKIN, kernel=EXPONENTIAL, ell=1.0):
    """Unit cube, p=2, 8^3 elements (N = 1000), M = 10 (FP64-oracle case)."""
    return problem(method, "cube", 2, (8, 8, 8), kernel, ell, M=10, block=16,
                   name=f"cube_p2_8^3_{kernel}_l{ell:g}_{method}")


def cube_p3_20(method=GALERKIN, kernel=GAUSSIAN, ell=None, precision="fp32"):
    """Unit cube, p=3, 20^3 elements (N = 12167), M = 50, b = 16."""
    if ell is None:
        ell = 0.5 if kernel == GAUSSIAN else 1.0
    return problem(method, "cube", 3, (20, 20, 20), kernel, ell, M=50, block=16, precision=precision,
                   name=f"cube_p3_20^3_{kernel}_l{ell:g}_{method}")


def annulus_p4(method=GALERKIN, kernel=GAUSSIAN, ell=None, precision="fp32", nel=(32, 32, 16)):
    """Quarter annulus r in [1,2], height 1, p=4, 32x32x16 elements (N = 25920), M = 100, b = 32."""
    if ell is None:
        ell = 0.5 if kernel == GAUSSIAN else 0.25
    return problem(method, "quarter_annulus", 4, nel, kernel, ell, M=100, block=32,
                   precision=precision, r0=1.0, r1=2.0, height=1.0,
                   name=f"annulus_p4_{nel[0]}x{nel[1]}x{nel[2]}_{kernel}_l{ell:g}_{method}")


def cube_p2_64(method=GALERKIN, precision="fp32"):
    """Unit cube, p=2, 64^3 elements (N = 287496), Gaussian l=0.2, M = 200, b = 64."""
    return problem(method, "cube", 2, (64, 64, 64), GAUSSIAN, 0.2, M=200, block=64, precision=precision,
                   name=f"cube_p2_64^3_gaussian_l0.2_{method}")


def nurbs_annulus_net(r0=1.0, r1=2.0, height=1.0):
    """Control net of the quarter annulus as a general NURBS volume: the
    rational quadratic quarter circle (control points (1,0), (1,1), (0,1),
    weights 1, 1/sqrt(2), 1) along xi, linear in the radius (eta) and in z
    (zeta).  Same map as the closed-form quarter annulus."""
    w = (1.0, 1.0 / math.sqrt(2.0), 1.0)
    cx, cy = (1.0, 1.0, 0.0), (0.0, 1.0, 1.0)
    ctrl = np.zeros((2, 2, 3, 4))
    for j3 in range(2):
        for j2, r in enumerate((r0, r1)):
            for j1 in range(3):
                ctrl[j3, j2, j1] = (r * cx[j1], r * cy[j1], height * j3, w[j1])
    return dict(degree=(2, 1, 1), knots=([0, 0, 0, 1, 1, 1], [0, 0, 1, 1], [0, 0, 1, 1]), ctrl=ctrl)


def half_cylinder_net(r0=8.0, r1=10.0, length=15.0):
    """Control net of a thick-walled half cylinder as one NURBS patch: along
    xi the half circle as two rational quadratic quarter arcs (knots
    0,0,0,1/2,1/2,1,1,1; control points (1,0), (1,1), (0,1), (-1,1), (-1,0)
    with weights 1, 1/sqrt(2), 1, 1/sqrt(2), 1), so the map is only C^0 in
    the knot sense at xi = 1/2; linear in the radius (eta, r0..r1) and along
    the axis (zeta, 0..length)."""
    s = 1.0 / math.sqrt(2.0)
    w = (1.0, s, 1.0, s, 1.0)
    cx, cy = (1.0, 1.0, 0.0, -1.0, -1.0), (0.0, 1.0, 1.0, 1.0, 0.0)
    ctrl = np.zeros((2, 2, 5, 4))
    for j3 in range(2):
        for j2, r in enumerate((r0, r1)):
            for j1 in range(5):
                ctrl[j3, j2, j1] = (r * cx[j1], r * cy[j1], length * j3, w[j1])
    return dict(degree=(2, 1, 1), knots=([0, 0, 0, 0.5, 0.5, 1, 1, 1], [0, 0, 1, 1], [0, 0, 1, 1]), ctrl=ctrl)


# The paper's numerical examples (Sec. 4) on the half cylinder: element counts
# (circumferential, radial, axial).  Example 1 (exponential kernel, p = 2,
# h-refinement): the five meshes that reproduce Table 1's N (and Ntilde for
# Cases 2-5) under the C^0-line rule; Example 2 (Gaussian kernel,
# k-refinement): the Case 1 mesh with p = 2..6 (Table 2).  The correlation
# length 5 is used throughout; the dimensions r0 = 8, r1 = 10, length 15 are
# a fit to the mesh sizes h of Table 1 read as element diagonals.
HALF_CYLINDER = dict(r0=8.0, r1=10.0, length=15.0, ell=5.0)
HALF_CYLINDER_EXAMPLE1 = [(32, 1, 8), (28, 2, 15), (32, 2, 18), (38, 2, 21), (42, 3, 23)]
HALF_CYLINDER_EXAMPLE2 = [(p, (32, 1, 8)) for p in (2, 3, 4, 5, 6)]


def kinked_box_net(kink=0.5, at=0.3, hi=(1.0, 1.0, 1.0)):
    """The box [0, hi] as a NURBS patch whose xi direction is piecewise
    linear: parameter `kink` maps to x = at * hi[0], so dx/dxi (and |det DF|)
    jumps there, a C^0 line.  Linear in eta and zeta, unit weights."""
    ctrl = np.zeros((2, 2, 3, 4))
    for j3 in range(2):
        for j2 in range(2):
            for j1, x in enumerate((0.0, at * hi[0], hi[0])):
                ctrl[j3, j2, j1] = (x, hi[1] * j2, hi[2] * j3, 1.0)
    return dict(degree=(1, 1, 1), knots=([0, 0, kink, 1, 1], [0, 0, 1, 1], [0, 0, 1, 1]), ctrl=ctrl)


def nurbs_blob_net(seed=0, n=(4, 4, 4), degree=(2, 2, 2), wiggle=0.06, wrange=(0.6, 1.6)):
    """Seeded curved volume near the unit cube: open uniform knots with
    n[k] - degree[k] spans, control points at the knot averages (Greville
    abscissae) each moved by up to `wiggle` per coordinate (faces included),
    weights drawn independently per control point in `wrange` (so they are
    not a tensor product)."""
    rng = np.random.default_rng(seed)
    knots, grev = [], []
    for k in range(3):
        p, m = int(degree[k]), int(n[k])
        nel = m - p
        t = [0.0] * (p + 1) + [e / nel for e in range(1, nel)] + [1.0] * (p + 1)
        knots.append(t)
        grev.append([sum(t[i + 1:i + p + 1]) / p for i in range(m)])
    g3, g2, g1 = np.meshgrid(grev[2], grev[1], grev[0], indexing="ij")
    xyz = np.stack([g1, g2, g3], axis=-1) + rng.uniform(-wiggle, wiggle, g1.shape + (3,))
    w = rng.uniform(wrange[0], wrange[1], g1.shape + (1,))
    return dict(degree=tuple(int(d) for d in degree), knots=tuple(knots), ctrl=np.concatenate([xyz, w], axis=-1))


def normal_block(seed, n, b, dtype=np.float64):
    """Seeded N(0, 1) block of shape (n, b)."""
    return np.random.default_rng(seed).standard_normal((n, b)).astype(dtype)


def uniform_points(seed, n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Seeded uniform points in a box, shape (n, 3), FP64."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + (hi - lo) * rng.random((n, 3))


def tensor_grid_points(counts, domain="cube"):
    """Tensor grid of counts[0] x counts[1] x counts[2] points with the first
    direction fastest (the order of the problems' point sets), evenly spaced in
    the parameters, shape (n, 3), FP64.  domain "cube": the unit cube.
    "quarter_annulus": angle 0..pi/2 (first direction), radius 1..2, height
    0..1."""
    u = [np.linspace(0.0, 1.0, int(c)) for c in counts]
    w, v, t = np.meshgrid(u[2], u[1], u[0], indexing="ij")
    t, v, w = t.ravel(), v.ravel(), w.ravel()
    if domain == "cube":
        return np.stack([t, v, w], axis=1)
    if domain == "quarter_annulus":
        r, th = 1.0 + v, 0.5 * math.pi * t
        return np.stack([r * np.cos(th), r * np.sin(th), w], axis=1)
    raise ValueError(domain)


SERVING_SEED = 210100629


def serving_stream(n_requests=512, seed=SERVING_SEED, mean_interarrival=1.0, max_pairs=None,
                   pair_count=None, nmin=8, nmax=40):
    """Request stream: seed-drawn mesh n^3 (cube) or n x n x ceil(n/2)
    (annulus), p in {2,3,4}, domain, kernel and method uniform over their two
    options, ell ~ U[0.1, 2], M ~ U{10..100}, b = 16 for M <= 50 else 32,
    Poisson arrivals with the given mean inter-arrival time.

    `pair_count(desc) -> float` and `max_pairs` let the caller resample
    requests whose kernel-pair count per block product exceeds a cap."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while len(out) < n_requests:
        n = int(rng.integers(nmin, nmax + 1))
        p = int(rng.integers(2, 5))
        domain = ["cube", "quarter_annulus"][int(rng.integers(0, 2))]
        kernel = [GAUSSIAN, EXPONENTIAL][int(rng.integers(0, 2))]
        method = [GALERKIN, COLLOCATION][int(rng.integers(0, 2))]
        ell = float(rng.uniform(0.1, 2.0))
        M = int(rng.integers(10, 101))
        gap = float(rng.exponential(mean_interarrival))
        nel = (n, n, n) if domain == "cube" else (n, n, int(math.ceil(n / 2)))
        kw = dict(r0=1.0, r1=2.0, height=1.0) if domain == "quarter_annulus" else {}
        d = problem(method, domain, p, nel, kernel, ell, M=M, block=16 if M <= 50 else 32, **kw)
        if max_pairs is not None and pair_count is not None and pair_count(d) > max_pairs:
            continue
        t += gap
        d["arrival"] = t
        d["id"] = len(out)
        out.append(d)
    return out
