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


def normal_block(seed, n, b, dtype=np.float64):
    """Seeded N(0, 1) block of shape (n, b)."""
    return np.random.default_rng(seed).standard_normal((n, b)).astype(dtype)


def uniform_points(seed, n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Seeded uniform points in a box, shape (n, 3), FP64."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + (hi - lo) * rng.random((n, 3))


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
