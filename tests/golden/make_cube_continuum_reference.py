"""Writes tests/golden/cube_continuum_spectra.json: the 20 largest eigenvalues
of the continuous K-L integral operators on the unit cube that the method
comparison of bench.py (--compare) measures against:

- L1-exponential kernel, ell = 1: exact, products of the univariate
  closed-form eigenvalues (oracle.analytic, Ghanem & Spanos form);
- Gaussian kernel, ell = 0.5: products of univariate eigenvalues from a fine
  FP64 discretisation (oracle.product1d, degree 6, 120 elements), converged to
  about 1e-12 relative for the indices involved.

Run from the repository root:  python tests/golden/make_cube_continuum_reference.py
"""
import json
import os
import sys

import numpy as np
import scipy.linalg as sla

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import analytic, product1d  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube_continuum_spectra.json")


def main(M=20):
    exp = analytic.exponential_box(M, 1.0)
    A, Z = product1d.galerkin_pencil_1d(6, 120, "gaussian", 0.5)
    l1 = np.sort(sla.eigh(A, Z, eigvals_only=True))[::-1][:40]
    P = (l1[:, None, None] * l1[None, :, None] * l1[None, None, :]).ravel()
    gau = np.sort(P)[::-1][:M]
    rec = {"what": "20 largest eigenvalues of the continuous covariance operators on the unit cube, sigma = 1",
           "script": "tests/golden/make_cube_continuum_reference.py",
           "exponential_l1": {"source": "oracle.analytic.exponential_box (closed form)", "lambda": exp.tolist()},
           "gaussian_l0.5": {"source": "oracle.product1d univariate Galerkin, p=6, 120 elements",
                             "lambda": gau.tolist()}}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
