"""Writes tests/golden/annulus_p4_32x32x16_gaussian_l0.5_galerkin.json: the 100
largest eigenvalues of the Galerkin-IBQ discretisation (paper Sec. 3.1) on the
quarter annulus r in [1, 2], height 1, p = 4, 32 x 32 x 16 elements (N = 25920),
Gaussian kernel with ell = 0.5, sigma = 1, computed with the FP64 oracle only:
the nine-step operator of oracle.galerkin with its kernel product done by the
plain C/OpenMP FP64 oracle (oracle/cmatvec.c), and ARPACK (scipy eigsh) on the
symmetric standard form A' = L^-1 A L^-T.

Run from the repository root:  python tests/golden/make_annulus_reference.py
(about 10-20 minutes on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np
from scipy.sparse.linalg import LinearOperator, eigsh

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cmatvec, galerkin, geometry  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "annulus_p4_32x32x16_gaussian_l0.5_galerkin.json")


def main(M=100):
    dom = geometry.QuarterAnnulus(1.0, 2.0, 1.0)
    g = galerkin.GalerkinIBQ(dom, 4, (32, 32, 16), "gaussian", 0.5, sigma=1.0)
    print("N", g.N, "Ntilde", g.Nt, flush=True)

    def gamma_apply(Y):
        return cmatvec.gamma_apply("gaussian", 1.0, 0.5, g.X, g.X, Y)

    count = [0]
    t0 = time.time()

    def matvec(v):
        count[0] += 1
        if count[0] % 25 == 0:
            print(f"  matvec {count[0]}  {time.time() - t0:.0f} s", flush=True)
        return g.apply_Aprime(v.reshape(-1, 1), gamma_apply=gamma_apply)[:, 0]

    op = LinearOperator((g.N, g.N), matvec=matvec, dtype=np.float64)
    v0 = np.random.default_rng(0).standard_normal(g.N)
    lam = eigsh(op, k=M, which="LA", ncv=2 * M + 20, tol=1e-13, v0=v0, return_eigenvectors=False)
    lam = np.sort(lam)[::-1]
    rec = {
        "what": "100 largest generalized eigenvalues, Galerkin-IBQ, quarter annulus r in [1,2], height 1, "
                "p=4, 32x32x16 elements, C^{p-1} interpolation space, Gaussian kernel exp(-|x-y|^2/0.5^2), "
                "sigma=1",
        "source": "oracle.galerkin.GalerkinIBQ nine-step operator (FP64) + oracle/cmatvec.c kernel product + "
                  "scipy ARPACK eigsh, tol 1e-13",
        "script": "tests/golden/make_annulus_reference.py",
        "N": g.N,
        "matvecs": count[0],
        "seconds": time.time() - t0,
        "lambda": lam.tolist(),
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", OUT, "matvecs", count[0], flush=True)


if __name__ == "__main__":
    main()
