"""FP64 CPU oracle for the matrix-free isogeometric Karhunen-Loeve hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of what the paper "A comparison of matrix-free isogeometric
Galerkin and collocation methods for Karhunen-Loeve expansion" (Mika,
Hiemstra, Hughes, Schillinger) computes.  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
library never does, and this package never imports the product.

Modules
-------
splines      knot vectors, Cox-de Boor basis, Greville abscissae, Gauss rules,
             univariate mass / mixed-mass / collocation matrices (Sec. 3.1).
geometry     parametric-to-physical maps F and |det DF| (cube, quarter annulus).
kernels      covariance kernels Gamma(x, x').
kron         action of Kronecker-product matrices (definition of the product).
galerkin     matrix-free Galerkin with interpolation based quadrature (Sec. 3.1,
             eq. for A = M^T B~^-1 J Gamma J B~^-T M) and standard Gauss
             quadrature Galerkin (Sec. 3.1, eq. galerkin_system_matrices).
collocation  isogeometric collocation (Sec. 3.2, eq. colloc_system_matrices,
             Algorithm 1).
product1d    exact spectra of separable kernels on boxes as products of 1D
             pencils.
extruded     exact spectra of separable kernels on extruded domains (box,
             quarter annulus) as products of a cross-section pencil and a 1D
             pencil along the extrusion.
analytic     closed-form eigenpairs of the 1D exponential kernel.
errors       eigenvalue error measures (Sec. 4.1, eps_i and mean eps).
cmatvec      ctypes wrapper of the plain C OpenMP FP64 Gamma-times-block product.
"""
