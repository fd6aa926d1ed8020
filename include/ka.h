/* ka.h -- C ABI of the MI355X matrix-free isogeometric Karhunen-Loeve library.
 *
 * The library computes the leading eigenpairs of the generalized eigenvalue
 * problem  A v = lambda Z v  (paper Sec. 1, eq. matrix_equations) that the
 * Galerkin (Sec. 3.1) and collocation (Sec. 3.2) discretisations of the
 * Fredholm problem (Sec. 2, eq. fredholm) produce, without ever forming the
 * dense matrix A.  The hot path is the on-the-fly covariance-kernel product
 * Gamma * Y inside the standard-form operator A' (Sec. 3, eq. standard).
 *
 * Conventions
 * -----------
 * - Tensor index of a degree of freedom: i = i1 + n1 * (i2 + n2 * i3), so the
 *   Kronecker factors read Z = Z3 (x) Z2 (x) Z1 (Sec. 3.1).
 * - Blocks of vectors are column-major FP64, N rows, leading dimension ld >= N.
 * - Pointers named *_dev are device pointers (hipMalloc / torch CUDA tensors);
 *   *_host are host pointers.  The caller owns every pointer it passes.
 * - Streams are hipStream_t passed as void* (NULL = the default stream).
 * - Return value: 0 = KA_OK, < 0 hard error (see ka_last_error()), > 0 soft
 *   condition (KA_NOT_CONVERGED).
 * - Device memory: ka_setup allocates the operator's arrays and workspace;
 *   ka_apply_A, ka_solve_Z, ka_gamma_apply and ka_gamma_apply_static
 *   allocate nothing (they are asynchronous on the given stream).  ka_eigs
 *   allocates its workspace on the first call and keeps it with the problem:
 *   a later call allocates only when it needs more (larger M), and then
 *   replaces the buffer.  ka_kl_sample keeps its own workspace the same way.
 *   ka_destroy frees everything.  ka_eigs is synchronous on the problem's
 *   stream.
 * - A problem handle must not be used from two host threads at once.
 */
#ifndef KA_H
#define KA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define KA_OK 0
#define KA_ERR_ARG (-1)       /* invalid argument or shape                  */
#define KA_ERR_OOM (-2)       /* device allocation failed                   */
#define KA_ERR_HIP (-3)       /* a HIP runtime call or launch failed         */
#define KA_ERR_SINGULAR (-4)  /* a factorisation met a (near) zero pivot     */
#define KA_ERR_STATE (-5)     /* call not valid for this problem / server    */
#define KA_NOT_CONVERGED 1    /* ka_eigs: maxit reached; partial results    */

/* ---- enumerations ------------------------------------------------------ */
enum ka_method { KA_GALERKIN_IBQ = 0,   /* Galerkin with interpolation-based quadrature (Sec. 3.1) */
                 KA_COLLOCATION = 1,    /* isogeometric collocation (Sec. 3.2, Algorithm 1)        */
                 KA_GALERKIN_GAUSS = 2  /* standard Galerkin with Gauss quadrature (Sec. 3.1, the
                                           method IBQ replaces): same trial space and Z as IBQ,
                                           Gamma between all quadrature points                   */ };
enum ka_domain { KA_BOX = 0, KA_QUARTER_ANNULUS = 1, KA_NURBS = 2 /* general single-patch NURBS volume */ };
enum ka_kernel { KA_GAUSSIAN = 0, /* sigma^2 exp(-|x-y|_2^2 / ell^2) */
                 KA_EXP_L1 = 1    /* sigma^2 exp(-|x-y|_1 / ell)     */ };
enum ka_precision { KA_FP32 = 0,  /* FP32 kernel tiles, FP32 MFMA contraction        */
                    KA_BF16X3 = 1 /* FP32 tiles split hi+lo into BF16, 3 BF16 MFMAs,
                                     FP32 accumulation                               */ };
enum ka_form { KA_A = 0,          /* the covariance matrix A itself                  */
               KA_APRIME = 1      /* the standard-form operator A' (Sec. 3, eq. standard):
                                     Galerkin L^-1 A L^-T, collocation Z^-1 A         */ };
enum ka_solve_op { KA_ZINV = 0,   /* X <- Z^-1 X                                     */
                   KA_LINV = 1,   /* X <- L^-1 X   (Galerkin, Z = L L^T)             */
                   KA_LTINV = 2   /* X <- L^-T X   (Galerkin)                        */ };

/* ---- problem description (paper Sec. 3; Sec. 4 for the spaces) ---------
 * method       KA_GALERKIN_IBQ (Sec. 3.1), KA_COLLOCATION (Sec. 3.2) or
 *              KA_GALERKIN_GAUSS (standard Galerkin, nq Gauss points per element
 *              and direction on both sides of Gamma: O((N_e nq^3)^2) pairs).
 * domain       KA_BOX: [lo, hi] (affine map); KA_QUARTER_ANNULUS: radii r0 < r1,
 *              quarter circle in the x-y plane extruded to `height` (exact
 *              rational quadratic NURBS map); KA_NURBS: the single-patch NURBS
 *              volume of geo_* below (Sec. 3.2), any positive weights.
 *              The analysis spaces live on the parametric cube [0,1]^3 with
 *              their own uniform knots (degree/nel); for the usual isogeometric
 *              setting those knots refine the geometry's.
 *              Collocation on KA_NURBS uses the rational trial space spanned by
 *              B_j / W (W the geometry's weight function, B_j the degree/nel
 *              B-splines): the span of the NURBS functions w_j B_j / W, so the
 *              eigenvalues are those of the NURBS basis, and the eigenvectors
 *              are coefficients of B_j / W.  Its collocation matrix is
 *              diag(1/W(g)) (Z_3 x Z_2 x Z_1) with B-spline factors Z_k, so no
 *              full LU is formed.
 * degree/nel   B-spline degree and element count per parametric direction
 *              (solution space with C^{p-1} continuity, open uniform knots).
 *              C^0 lines (Sec. 4.1): on KA_NURBS, an interior geometry knot
 *              repeated at least geo_degree[k] times is a line where the map
 *              is only C^0 (e.g. where two patches meet).  It is added to the
 *              analysis mesh if it is not a uniform breakpoint, the solution
 *              space is C^0 there (all methods), and the IBQ interpolation
 *              space C^-1; its two interpolation points at the line are
 *              evaluated from their own sides (|det DF| jumps there).
 *              ka_desc_size gives the resulting N and Ntilde.
 * interp_cont  Galerkin only: continuity of the interpolation space S~;
 *              -1 = automatic: C^0 for KA_EXP_L1 (Sec. 4.1), C^{p-1} for
 *              KA_GAUSSIAN (Sec. 4.2); otherwise 0 .. p-1 (C^-1 at C^0 lines
 *              in any case).
 * kernel/sigma/ell  covariance kernel and its parameters (ell > 0; ell = +inf
 *              is allowed for KA_GAUSSIAN and gives the constant kernel).
 * nq           collocation and Gauss Galerkin: Gauss points per element and
 *              direction (0 = p+1).
 * precision    contraction precision of the kernel product.
 * block        eigensolver block size b: 16, 32 or 64 (KA_ERR_ARG otherwise);
 *              also the largest nvec that one internal pass of ka_apply_A
 *              handles (larger nvec loops).
 * seed         seeds the eigensolver's start block.                          */
typedef struct ka_desc {
  int method;
  int domain;
  double lo[3], hi[3];
  double r0, r1, height;
  int degree[3];
  int nel[3];
  int interp_cont;
  int kernel;
  double sigma, ell;
  int nq;
  int precision;
  int block;
  unsigned long long seed;
  /* KA_NURBS only (ignored otherwise).  Host arrays, read during ka_setup,
   * ka_footprint and ka_server_submit (which copies them); not kept.
   * geo_degree[k] in 1..30 and geo_nctrl[k] >= geo_degree[k] + 1 control
   * points per direction; geo_knots: the three knot vectors one after the
   * other, geo_nctrl[k] + geo_degree[k] + 1 values each, non-decreasing and
   * open on [0, 1]; geo_ctrl: geo_nctrl[0] * geo_nctrl[1] * geo_nctrl[2]
   * control points as (x, y, z, weight), weight > 0, index j1 fastest.
   * Invalid data: KA_ERR_ARG. */
  int geo_degree[3];
  int geo_nctrl[3];
  const double* geo_knots;
  const double* geo_ctrl;
} ka_desc;

/* eigensolver report */
typedef struct ka_info {
  int iterations;        /* restart cycles                                     */
  int matvecs;           /* block applications of A'                           */
  int converged;         /* leading pairs meeting the tolerance                */
  int nev_computed;      /* M extended to the end of its eigenvalue cluster    */
  double max_residual;   /* max over the first M of |A'x - theta x| / max(|theta|, 1e-2 |theta_1|) */
  double max_imag_rel;   /* collocation: max |Im lambda| / |lambda| over the first M */
  double seconds;        /* wall time of the solve                             */
  double gamma_seconds;  /* device time inside the kernel-product launches     */
  double pairs;          /* kernel pair evaluations performed                  */
  int lambda_doubles;    /* doubles written to lambda_host: M, or 2M (collocation) */
  int floor_accepted;    /* of the first M pairs, those accepted only through the
                            arithmetic noise floor nu |theta_1| (residual above
                            tol max(|theta|, 1e-2 |theta_1|)); see ka_eigs      */
} ka_info;

typedef struct ka_problem ka_problem;

/* Build a problem: host FP64 setup of knots, Greville points, Gauss rules,
 * univariate mass / mixed-mass / collocation matrices and their factors
 * (Sec. 3.1, Z = Z3 x Z2 x Z1 and its Cholesky factors; Sec. 3.2 pivoted LU of
 * the Kronecker factors of Z, remark in Sec. 3.3), physical point sets, and
 * upload.  Allocates all device workspace.  `stream` becomes the problem's
 * stream for ka_eigs.  On error *out is NULL. */
int ka_setup(const ka_desc* desc, void* stream, ka_problem** out);

/* Sizes of the discretisation (Sec. 3.1: N trial functions, Ntilde points of
 * the interpolation space S~ at which Gamma is evaluated; Sec. 3.2: N
 * collocation points and the quadrature points of Algorithm 1): N degrees of
 * freedom, Ntilde IBQ interpolation points (0 for the other methods), Nquad
 * quadrature points (collocation and Gauss Galerkin; 0 for IBQ), and the device
 * bytes the problem holds now (set-up arrays, plus the eigensolver and K-L
 * sampling workspaces once allocated).  Any output pointer may be NULL. */
int ka_size(const ka_problem* p, int64_t* N, int64_t* Ntilde, int64_t* Nquad,
            size_t* device_bytes);

/* The sizes ka_size would report for a problem set up from `desc` (see
 * degree/nel and the C^0 lines in ka_desc); host only, no device work.
 * KA_ERR_ARG for an invalid description.  Any output pointer may be NULL. */
int ka_desc_size(const ka_desc* desc, int64_t* N, int64_t* Ntilde, int64_t* Nquad);

/* Device bytes ka_setup would allocate for `desc` (admission control); no
 * device work. */
int ka_footprint(const ka_desc* desc, size_t* device_bytes);

/* Y = A X or Y = A' X for nvec columns (device, column-major FP64).
 * Galerkin (Sec. 3.1): A = M^T B~^-1 J Gamma J B~^-T M, and A' = L^-1 A L^-T is
 * the nine-step product (L^-T, M, B~^-T, J, Gamma, J, B~^-1, M^T, L^-1).
 * Collocation (Sec. 3.2, Algorithm 1): A = Gamma_c diag(J W) R_q, A' = Z^-1 A.
 * X and Y must not overlap.  Async on `stream`; no allocation. */
int ka_apply_A(ka_problem* p, int form, const double* X_dev, int64_t ldx,
               double* Y_dev, int64_t ldy, int nvec, void* stream);

/* In-place FP64 Kronecker solves on nvec columns (device, column-major):
 * KA_ZINV X <- Z^-1 X (Galerkin: mass matrix; collocation: Z_ij = R_j(x_i)),
 * KA_LINV X <- L^-1 X, KA_LTINV X <- L^-T X (Galerkin only; else KA_ERR_STATE).
 * Galerkin (Sec. 3.1): Z = Z3 (x) Z2 (x) Z1 is the mass matrix of the trial
 * space B_i / sqrt|det DF| (eq. trialspace), Z = L L^T with L = L3 (x) L2 (x) L1
 * from the Cholesky factors of the Z_k; A' = L^-1 A L^-T and v = L^-T v'.
 * Collocation (Sec. 3.2): Z_ij = R_j(x_i); the paper factors P Z Q = L U with
 * complete pivoting; here Z is the Kronecker product of its univariate factors
 * (remark in Sec. 3.3), each LU-factored with partial pivoting in FP64, equal
 * in exact arithmetic (on KA_NURBS also scaled by diag(1/W), see ka_desc).
 * Applied as FP64 mode products with the inverse factors.  X: ld >= N.
 * Async on `stream`; no allocation. */
int ka_solve_Z(ka_problem* p, int op, double* X_dev, int64_t ld, int nvec, void* stream);

/* Leading M eigenpairs of the generalized problem A v = lambda Z v (Sec. 1,
 * eq. matrix_equations), solved in the standard form A' v' = lambda v',
 * v = C v' (Sec. 3, eq. standard; Galerkin C = L^-T, collocation C = I), by a
 * block Krylov method with thick restarts (FP64 basis, orthogonalisation and
 * Rayleigh-Ritz on the device; the paper leaves the iterative solver open).
 * Stops when, for the first M Ritz pairs (M extended to the end of its
 * cluster), |A'x - theta x| <= max(tol |theta|, max(1e-2 tol, nu) |theta_1|),
 * where nu is the arithmetic noise floor of the operator (Galerkin: 4e-6 FP32,
 * 1e-4 BF16x3; collocation: 2e-7 FP32, 5e-6 BF16x3).  A Galerkin pair with
 * |theta| > nu |theta_1| accepted only through that floor must also satisfy
 * r^2 / gap <= 0.1 tol max(|theta|, 1e-2 |theta_1|) (gap: distance to the
 * nearest Ritz value that r and nu can separate from theta); pairs below the
 * floor carry an absolute error of order nu |theta_1|.  Collocation's A' is
 * not symmetric and its eigenvalue error is first order in the residual: a
 * collocation pair accepted only through the floor must also have moved by
 * at most 0.1 tol max(|theta|, 1e-2 |theta_1|) since the previous
 * Rayleigh-Ritz step (never in the first restart cycle).
 * info->floor_accepted counts the pairs accepted through the floor (either
 * method).  Also stops after maxit restart cycles,
 * or after three cycles without a 10% drop of the largest scaled residual
 * (both return KA_NOT_CONVERGED; results are still written).
 * lambda_host: host array of lambda_len doubles; the solve writes M doubles
 *   (Galerkin methods), or 2M doubles re/im interleaved (collocation), sorted
 *   by descending real part (info->lambda_doubles says which).  KA_ERR_ARG,
 *   before any device work, if lambda_len is smaller.
 * Workspace: about (2 m + 4 (M + b + 1)) N doubles (m the Krylov basis width:
 *   M + b plus at least two blocks), allocated on the first call and kept by
 *   the problem (see the conventions above).
 * V_dev: N x M column-major device array or NULL.  Galerkin eigenvectors are
 *   Z-orthonormal (v = L^-T v'); collocation eigenvectors have unit 2-norm (a
 *   complex pair is stored as real part, imaginary part in consecutive
 *   columns).  Each vector's largest-magnitude entry is made positive.
 * info may be NULL.  Synchronous. */
int ka_eigs(ka_problem* p, int M, double tol, int maxit, double* lambda_host, int64_t lambda_len,
            double* V_dev, ka_info* info);

/* The raw fused kernel product (hot path, paper Sec. 3.1 step Gamma and
 * Algorithm 1 step 3): Z[i, :] = sigma^2 sum_c Gamma(xr_i, xc_c) Y[c, :].
 * xr: nr x 3, xc: nc x 3 FP32 row-major physical coordinates; Y: nc x b and
 * Z: nr x b FP32 row-major (point-major, b contiguous); b in {16, 32, 64}.
 * precision KA_FP32 or KA_BF16X3.  Scratch from `work_dev` (work_bytes,
 * 16-byte aligned): the split-K partial sums (nsplit * nr * b * 4 bytes when
 * the columns are split) and, for KA_BF16X3, Y split into hi/lo BF16 parts
 * (ceil(nc / 64) * 64 * b * 4 bytes); pass ka_gamma_workspace() bytes.
 * Async on `stream`. */
int ka_gamma_apply(int kernel, double sigma, double ell, const float* xr_dev, int64_t nr,
                   const float* xc_dev, int64_t nc, const float* Y_dev, int b, float* Z_dev,
                   int precision, void* work_dev, size_t work_bytes, void* stream);

/* Scratch bytes ka_gamma_apply needs for these sizes. */
size_t ka_gamma_workspace(int64_t nr, int64_t nc, int b, int precision);

/* ka_gamma_apply without any device allocation and without a workspace
 * argument, for callers that cannot allocate device memory (code under HIP
 * stream capture, serving loops and harnesses that forbid hipMalloc).  Same
 * arguments, kernels and results as ka_gamma_apply; its scratch is a
 * file-scope device array of ka_gamma_static_capacity() bytes (128 MiB), one
 * per GPU, held until the process ends and looked up on the first call on each
 * device.  A product whose ka_gamma_workspace() exceeds that capacity fails
 * with KA_ERR_ARG before anything is launched.  All calls on one GPU share the
 * array: calls that overlap on the device (concurrent streams) race and must
 * be serialised by the caller.  Nothing in the array needs clearing: every
 * entry a call reads is written earlier in the same call.  Async on `stream`. */
int ka_gamma_apply_static(int kernel, double sigma, double ell, const float* xr_dev, int64_t nr,
                          const float* xc_dev, int64_t nc, const float* Y_dev, int b, float* Z_dev,
                          int precision, void* stream);
size_t ka_gamma_static_capacity(void);

/* ---- K-L field sampling (paper Sec. 2, eq. kle) --------------------------
 * Truncated expansion alpha_M(x, s) = mu + sum_{i<M} sqrt(lambda_i) phi_i(x) xi_i(s)
 * at the tensor grid of parametric points (grid[0][i1], grid[1][i2], grid[2][i3])
 * of the problem's domain, for nsamples draws.
 * phi_i: the eigenfunction with coefficient column i of V in the problem's
 *   trial space, as ka_eigs returns V (Galerkin: v = L^-T v', phi = sum_j v_j
 *   B_j / sqrt|det DF|; collocation: phi = sum_j v_j R_j, R_j = B_j / W on a
 *   KA_NURBS volume), scaled here to unit L2(D) norm.  The norm is taken with
 *   a Gauss rule per element and direction: p + 1 points for the Galerkin
 *   methods (exact), the collocation rule's nq points for collocation.
 * lambda_host: M finite eigenvalues >= 0 (collocation: their real parts).
 * V_dev: N x M column-major FP64 (ldv >= N).  grid_host: npts[0] + npts[1] +
 *   npts[2] coordinates in [0, 1], direction 1 first.  xi_dev: M x nsamples
 *   column-major FP64 (ldxi >= M), the draws (N(0,1) for a Gaussian field).
 * field_dev: P x nsamples column-major FP64 (ldf >= P), P = npts[0] npts[1]
 *   npts[2], grid point index i1 + npts[0] (i2 + npts[1] i3).
 * Its device workspace (about (P + quadrature points) x M doubles) is kept
 * by the problem between calls, grown when a call needs more, and freed by
 * ka_destroy; collocation also keeps the quadrature data of the norms from
 * its first call.  Synchronizes `stream` before it returns.  Errors: KA_ERR_ARG (bad
 * sizes or values), KA_ERR_SINGULAR (an eigenfunction of zero norm),
 * KA_ERR_OOM, KA_ERR_HIP. */
int ka_kl_sample(ka_problem* p, int M, const double* lambda_host, const double* V_dev, int64_t ldv,
                 const int npts[3], const double* grid_host, int nsamples, const double* xi_dev,
                 int64_t ldxi, double mu, double* field_dev, int64_t ldf, void* stream);

/* Timing of kernel-product launches issued through a problem since the last
 * reset (HIP events on the launch stream; enabled by ka_profile_enable). */
int ka_profile_enable(ka_problem* p, int on);
int ka_profile_read(ka_problem* p, int* launches, double* total_ms, double* pairs);
int ka_profile_reset(ka_problem* p);

void ka_destroy(ka_problem* p);

/* ---- serving (continuous batching of K-L solve requests on one GPU) ----
 * Not in the paper: a request loop around the solver.  Requests queue in
 * arrival order; one is admitted once it has arrived (arrival_s, seconds
 * after the first ka_server_run), a slot is free and a contiguous range of its
 * device footprint (ka_request_bytes) is free in the server's arena.  The
 * arena is one device allocation of hbm_budget bytes made by
 * ka_server_create, with the dispatcher's launch lists beside it; a request's
 * problem and eigensolver workspace are laid out inside its range, so
 * serving allocates and frees no device memory between ka_server_create and
 * ka_server_destroy.  Admitted solves keep their Krylov state on the device,
 * each on its own stream; all their kernel products run together as shared
 * persistent launches, one block application per request per loop
 * iteration; a finished request returns its range at once so waiting ones
 * join the running batch.  A request's eigenvalues are bitwise the same
 * alone or in any mix (each product keeps its own split-K partition and
 * every reduction a fixed order). */
typedef struct ka_server ka_server;

typedef struct ka_result {
  int64_t id;            /* from ka_server_submit                              */
  uint64_t tag;          /* caller's tag                                       */
  int status;            /* ka_eigs return code, or KA_ERR_OOM if it can never fit */
  ka_info info;
  double arrival_s, admit_s, done_s;   /* seconds on the server clock           */
} ka_result;

/* hbm_budget: bytes of the device arena (allocated here; KA_ERR_OOM if that
 * fails); max_slots: requests solved at once (1..256). */
int ka_server_create(size_t hbm_budget, int max_slots, ka_server** out);
/* Device bytes a request holds while admitted: ka_footprint plus the
 * eigensolver workspace for M eigenpairs at the descriptor's block size. */
int ka_request_bytes(const ka_desc* desc, int M, size_t* bytes);
/* lambda_host: caller-owned, lambda_len doubles, at least M (Galerkin) or 2M
 * (collocation, re/im interleaved), written when the request completes
 * (KA_ERR_ARG at submission if too small).  tol/maxit as for ka_eigs. */
int ka_server_submit(ka_server* s, const ka_desc* desc, int M, double tol, int maxit, double arrival_s,
                     uint64_t tag, double* lambda_host, int64_t lambda_len, int64_t* req_id);
/* Serve until every submitted request has completed (or timeout_s elapses:
 * KA_NOT_CONVERGED).  Synchronous; may be called again after new submits. */
int ka_server_run(ka_server* s, double timeout_s);
/* Move up to max completed results into out; *n = number moved. */
int ka_server_poll(ka_server* s, ka_result* out, int max, int* n);
int ka_server_stats(ka_server* s, int* batches, double* mean_items, int* max_active, size_t* bytes_in_use);
void ka_server_destroy(ka_server* s);

/* Last error message of the calling host thread. */
const char* ka_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KA_H */
