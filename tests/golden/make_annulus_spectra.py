"""Writes tests/golden/annulus_p4_32x32x16_spectra.json: the leading eigenvalues
of the four discretisations of the curved-domain workload, computed with the
FP64 oracle only (oracle/extruded.py: products of the cross-section pencil and
the pencil along the extrusion, exact for the separable kernels on the
extruded quarter annulus).

Workload: quarter annulus r in [1, 2], height 1, p = 4, 32 x 32 x 16 elements
(N = 25920); Galerkin-IBQ (Sec. 3.1; C^{p-1} interpolation space for the
Gaussian kernel, C^0 for the exponential, 1,081,665 interpolation points) and
collocation (Sec. 3.2, Algorithm 1; (p+1)^3 Gauss points per element,
2,048,000 quadrature points); Gaussian kernel exp(-|x-y|_2^2 / 0.5^2) and
exponential kernel exp(-|x-y|_1 / 0.25), sigma = 1.

Run from the repository root:  python tests/golden/make_annulus_spectra.py
(under a minute on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import extruded, geometry  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "annulus_p4_32x32x16_spectra.json")
P, NEL = 4, (32, 32, 16)
ELL = {"gaussian": 0.5, "exponential": 0.25}
COUNT = 140   # M = 100 plus room for the end of a cluster and guard values


def main():
    ann = geometry.QuarterAnnulus(1.0, 2.0, 1.0)
    spectra = {}
    for method in ("galerkin", "collocation"):
        for kernel, ell in ELL.items():
            t0 = time.time()
            if method == "galerkin":
                lam = extruded.galerkin_spectrum(ann, P, NEL, kernel, ell, M=COUNT)
                rec = {"lambda": lam.tolist()}
            else:
                lam = extruded.collocation_spectrum(ann, P, NEL, kernel, ell, M=COUNT)
                rec = {"lambda": lam.real.tolist(), "max_abs_imag": float(np.abs(lam.imag).max())}
            rec["ell"] = ell
            spectra[f"{method}-{kernel}"] = rec
            print(f"{method}-{kernel}: lambda_1 = {lam[0].real:.12e}  ({time.time() - t0:.1f} s)", flush=True)
    out = {
        "what": f"{COUNT} leading generalized eigenvalues (descending real part), quarter annulus r in [1,2], "
                "height 1, p=4, 32x32x16 elements, sigma=1; Galerkin-IBQ and collocation, Gaussian "
                "exp(-|x-y|_2^2/0.5^2) and exponential exp(-|x-y|_1/0.25) kernels",
        "source": "oracle/extruded.py (FP64): products of the cross-section and extrusion pencils",
        "script": "tests/golden/make_annulus_spectra.py",
        "N": 25920,
        "spectra": spectra,
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
