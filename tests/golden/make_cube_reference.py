"""Writes tests/golden/cube_p3_20_reference_spectra.json: the 50 largest
eigenvalues of the four discretisations the benchmark solves on the unit cube
(p = 3, 20^3 elements): Galerkin-IBQ and collocation, each with the Gaussian
kernel (ell = 0.5, C^{p-1} interpolation space) and the L1-exponential kernel
(ell = 1, C^0 interpolation space), sigma = 1.  On the cube both kernels are
separable and every matrix is a Kronecker product, so the spectra are exact
products of univariate FP64 pencil eigenvalues (oracle.product1d).

Run from the repository root:  python tests/golden/make_cube_reference.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import product1d  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube_p3_20_reference_spectra.json")


def main(M=50):
    rec = {"what": "50 largest generalized eigenvalues, unit cube, p=3, 20^3 elements, sigma=1; "
                   "collocation at Greville points with (p+1)^3 Gauss points per element (real parts; the "
                   "univariate collocation spectra are real here)",
           "source": "oracle.product1d (products of univariate FP64 pencil eigenvalues)",
           "script": "tests/golden/make_cube_reference.py",
           "spectra": {}}
    for method in ("galerkin", "collocation"):
        for kernel, ell in (("gaussian", 0.5), ("exponential", 1.0)):
            if method == "galerkin":
                lam = product1d.galerkin_box_spectrum(3, (20, 20, 20), kernel, ell, M=M)
            else:
                lam = product1d.collocation_box_spectrum(3, (20, 20, 20), kernel, ell, M=M).real
            rec["spectra"][f"{method}-{kernel}"] = {"ell": ell, "lambda": [float(x) for x in lam]}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
