"""Writes tests/golden/cube_p2_64_reference_spectra.json: the 240 largest
eigenvalues of the large matrix-free workload, the unit cube with p = 2 and
64^3 elements (N = 287,496), Gaussian kernel exp(-|x-y|_2^2 / 0.2^2), sigma = 1:
Galerkin-IBQ (C^{p-1} interpolation space, 287,496 interpolation points) and
collocation ((p+1)^3 Gauss points per element, 7,077,888 quadrature points).
On the cube the kernel is separable and every matrix is a Kronecker product,
so the spectra are exact products of univariate FP64 pencil eigenvalues
(oracle.product1d).  240 values: M = 200 plus the rest of the cluster the
200th value falls in and guard values.

Run from the repository root:  python tests/golden/make_cube_p2_64_reference.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import product1d  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube_p2_64_reference_spectra.json")


def main(count=240):
    rec = {"what": f"{count} largest generalized eigenvalues, unit cube, p=2, 64^3 elements, Gaussian kernel "
                   "ell=0.2, sigma=1; collocation at Greville points with (p+1)^3 Gauss points per element (real "
                   "parts; the univariate collocation spectra are real here)",
           "source": "oracle.product1d (products of univariate FP64 pencil eigenvalues)",
           "script": "tests/golden/make_cube_p2_64_reference.py",
           "spectra": {}}
    lam = product1d.galerkin_box_spectrum(2, (64, 64, 64), "gaussian", 0.2, M=count)
    rec["spectra"]["galerkin-gaussian"] = {"ell": 0.2, "lambda": [float(x) for x in lam]}
    lam = product1d.collocation_box_spectrum(2, (64, 64, 64), "gaussian", 0.2, M=count)
    assert abs(lam.imag).max() == 0.0
    rec["spectra"]["collocation-gaussian"] = {"ell": 0.2, "lambda": [float(x) for x in lam.real]}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
