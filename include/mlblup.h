/*
 * mlblup.h -- C ABI of the multilevel spatial BLUP solve on AMD MI355X (gfx950).
 *
 * Method: J. E. Castrillon-Candas, "Spatial best linear unbiased prediction:
 * a computational mathematics approach for high dimensional massive
 * datasets", arXiv:1701.00285.  Observations Z = X beta + eps at N sites in
 * d dimensions, eps ~ N(0, C(theta)) with a Matern covariance C, X the
 * total-degree monomial design (Sec. 2).  A kd-tree (Sec. 3.1, algorithms
 * Rule / InitialTree / MakeTree) and a multilevel basis W orthogonal to
 * col(X) (Sec. 3.1 construction) turn the kriging system into the
 * well-conditioned C_W gamma_W = W Z with C_W = W C W^T (Sec. 5.2,
 * eqs. Spatial:eqn1-3), solved by a Krylov (PCG) iteration whose product is
 * the three-step W^T -> C -> W chain (Sec. 6.2).
 *
 * Conventions for every entry point:
 *   - Return value is a status code (MLBLUP_OK = 0, negative on error); the
 *     message of the last error on the calling thread is mlblup_last_error().
 *   - "_host" pointers are host memory, "_dev" pointers are device memory of
 *     the current HIP device.  The caller owns every data buffer; the library
 *     never allocates device memory.  Sizes of the scratch it needs are
 *     reported by the *_workspace_bytes queries; the caller passes a device
 *     workspace of at least that size (256-byte aligned).
 *   - Device vectors of length N are in TREE ORDER (position k holds the
 *     point mlblup_tree_perm()[k] of the input).  Coordinates are row-major
 *     (point-major) N x d float64 arrays.
 *   - `stream` is a hipStream_t passed as void* (NULL = legacy default
 *     stream).  Device work is enqueued on it; calls that return scalars to
 *     the host (pcg_solve, blup_predict, blup_grad) synchronise it.
 *   - Handles (tree, basis) are immutable after construction and may be
 *     used from several streams at once; a workspace must not be shared by
 *     calls in flight at the same time.
 *   - Environment: MLBLUP_LOG_EVERY=k (k > 0) makes the Krylov solves print
 *     the recurrence residual every k iterations to stderr.
 */
#ifndef MLBLUP_H
#define MLBLUP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLBLUP_OK 0
#define MLBLUP_EINVAL (-1)     /* bad argument: shape, NULL, nu outside (0, 8] and not +inf, NaN input, small
                                  workspace */
#define MLBLUP_ERANK (-2)      /* design matrix rank < p on the point set (e.g. collinear points, duplicates) */
#define MLBLUP_ENOCONV (-3)    /* iteration limit reached; outputs hold the last iterate, info is filled */
#define MLBLUP_EBREAKDOWN (-4) /* Krylov breakdown: p.q <= 0 or a non-finite scalar */
#define MLBLUP_EHIP (-5)       /* HIP runtime error; the message names the call and the HIP error */
#define MLBLUP_ESTATE (-6)     /* handle not ready (e.g. basis used on device before mlblup_basis_upload) */

/* Arithmetic of the pair kernel (the dense covariance product). */
#define MLBLUP_FP64 0          /* FP64 differences, sqrt, exp, sums */
#define MLBLUP_FP32 1          /* FP32 kernel values: square products (N >= 16384) from FP32 coordinates relative
                                  to a block origin, FP32 sums over 16 columns then FP64; other products from
                                  FP64 squared distances with FP32 sqrt/exp and FP64 sums */
#define MLBLUP_MFMA_FP32 2     /* distance Gram on FP32 matrix cores, exact near tiles (8 <= d <= 32, half-integer
                                  nu, values only; elsewhere the MLBLUP_FP32 kernels) */
#define MLBLUP_MFMA_BF16X3 3   /* distance Gram on BF16 matrix cores with a hi/lo split (3 products); same scope */

/* Output selection bitmask of mlblup_cov_matvec. */
#define MLBLUP_VALUE 1         /* y  = C x            */
#define MLBLUP_DLOGRHO 2       /* dy = (rho dC/drho) x */

typedef struct mlblup_tree_s* mlblup_tree;
typedef struct mlblup_basis_s* mlblup_basis;
typedef struct mlblup_precond_s* mlblup_precond;

/* Preconditioner kinds (preconditioner remark of Sec. 5.2). */
#define MLBLUP_PREC_JACOBI 1   /* P_W = diag(C_W) */
#define MLBLUP_PREC_BLOCK 2    /* P_W = the diagonal blocks of C_W, one per cell (its own wavelets) */
#define MLBLUP_PREC_COARSE 3   /* the cell blocks of the finest level and one dense block of C_W over all
                                  coarser levels (a coarse space; not in the paper) */

/* mixed-precision schemes (mlblup_pcg_opts.mixed_scheme) */
#define MLBLUP_MIXED_FLEXIBLE 0
#define MLBLUP_MIXED_RELIABLE 1

/* Matern covariance sigma2 * phi(r; nu, rho), Definition in Sec. 3.1, rho > 0,
 * sigma2 > 0, z = sqrt(2 nu) r / rho:
 *   nu = 1/2, 3/2, 5/2: the half-integer closed forms, every precision and output;
 *   nu = +INFINITY: the Gaussian exp(-r^2 / (2 rho^2)) (the Definition's limit;
 *     the kernel of the accuracy experiment in Sec. 8), every precision and output;
 *   any other 0 < nu <= 8: values from a series at the origin and tables
 *     (entries below 1e-18 sigma2 dropped), FP64 or FP32 (the matrix-core
 *     precisions take the FP32 path); the rho-derivative sigma2 z^{nu+1}
 *     K_{nu-1}(z) from a second table; the preconditioners with FP32 values.
 *     Square FP64 value products use the symmetric kernel, the other general-nu
 *     products the row-tiled one. */
typedef struct {
  double nu;
  double rho;
  double sigma2;
} mlblup_matern;

/* Krylov solve options.  rtol: stop when |Z_W - C_W gamma_W|_2 <= rtol |Z_W|_2
 * on the UNPRECONDITIONED system, measured with the FP64 product (remark on
 * the stopping rule, Sec. 6.2).  precision: arithmetic of the inner product
 * (MLBLUP_FP64 runs plain PCG with a final FP64 residual check).  Lower
 * precisions keep vectors, dots and gamma_W in FP64 and use the
 * reduced-precision product inside the Krylov recurrence, in one of two
 * schemes (mixed_scheme):
 *   MLBLUP_MIXED_FLEXIBLE: flexible CG in FP64 (FP64 products) whose
 *     preconditioner is an inner PCG solve with the reduced-precision
 *     product to relative tolerance inner_rtol; refine_max bounds the outer
 *     steps.  Robust when cond(C_W) times the reduced precision's rounding
 *     unit exceeds 1.
 *   MLBLUP_MIXED_RELIABLE: one PCG recurrence with reduced-precision
 *     products; whenever its residual has fallen by the factor inner_rtol
 *     since the last check, the true FP64 residual replaces it and the
 *     search direction is kept (reliable updates); refine_max bounds the
 *     replacements.  Keeps the Krylov convergence of a single recurrence.
 * precond: NULL for P_W = I, else a preconditioner built and uploaded for
 * this basis (the paper's Jacobi P_W = diag(C_W), or its per-cell block
 * form).  history_host / history_cap: optional per-iteration record of the
 * recurrence residual. */
typedef struct {
  double rtol;
  int32_t max_iter;
  int32_t precision;
  int32_t refine_max;
  int32_t history_cap;           /* entries available in history_host (0 = no history) */
  double inner_rtol;
  mlblup_precond precond;        /* NULL: P_W = I; else an uploaded preconditioner of the same basis */
  double* history_host;          /* optional: |r_k| / |Z_W| after each Krylov iteration k (recurrence residual) */
  int32_t mixed_scheme;          /* MLBLUP_MIXED_FLEXIBLE or MLBLUP_MIXED_RELIABLE (ignored for MLBLUP_FP64) */
  double* state_dev;             /* MLBLUP_FP64 only, else ignored: NULL, or a device buffer of 2 (N - p) + 8
                                    doubles that receives the Krylov state (residual, search direction, r.z) when
                                    the solve returns, so that a later call can continue the same recurrence */
  int32_t resume;                /* with state_dev and use_x0 = 1 (gamma_W of the earlier call as the initial
                                    guess): continue the recurrence stored in state_dev instead of restarting it;
                                    the iterates are those of one uninterrupted solve */
} mlblup_pcg_opts;

typedef struct {
  int32_t inner_iters;    /* total Krylov iterations */
  int32_t outer_iters;    /* refinement steps (1 for a plain FP64 solve) */
  int32_t fp64_matvecs;   /* FP64 C_W products (iterations + residual checks) */
  int32_t lowp_matvecs;   /* reduced-precision C_W products */
  double relres_fp64;     /* final |Z_W - C_W gamma_W| / |Z_W| with the FP64 product */
  double zw_norm;         /* |Z_W|_2 */
} mlblup_pcg_info;

const char* mlblup_last_error(void);
int32_t mlblup_version(void);

/* ---- kd-tree (Sec. 3.1, algorithms Rule / InitialTree / MakeTree) ----------
 * Splits each cell on the coordinate axis of maximal variance of its points
 * at the median: points ordered by (coordinate, input index), the first
 * ceil(m/2) go left.  A cell with <= leaf_max points is a leaf.  Nodes are
 * numbered in preorder (root 0).  Inside a leaf, points are listed by input
 * index.  pts_host: n x d row-major float64 (copied).  n >= 1, 1 <= d <= 64,
 * leaf_max >= 1.  Non-finite coordinates -> MLBLUP_EINVAL. */
int mlblup_build_tree(const double* pts_host, int64_t n, int32_t d, int32_t leaf_max, mlblup_tree* out);
int mlblup_tree_info(mlblup_tree t, int64_t* n, int32_t* d, int32_t* n_nodes, int32_t* max_depth);
/* perm_host[k] = input index of the point at tree position k (n entries). */
int mlblup_tree_perm(mlblup_tree t, int64_t* perm_host);
/* Node arrays (n_nodes entries each; any pointer may be NULL): point range
 * [begin, end) in tree order, depth, split axis (-1 for leaves), children
 * (-1 for leaves), threshold (largest left coordinate; 0 for leaves). */
int mlblup_tree_nodes(mlblup_tree t, int64_t* begin, int64_t* end, int32_t* depth, int32_t* axis,
                      int32_t* left, int32_t* right, double* threshold);
void mlblup_tree_free(mlblup_tree t);

/* ---- multilevel basis (Sec. 3.1 construction; operators W, L, P) ---------
 * Bottom-up over the tree: for each cell the candidate vectors (leaf: unit
 * vectors of its points; internal: the children's scaling vectors) are
 * split by an orthogonal V into a scaling part spanning the range of
 * M^T (M = X^T V_cand, moments against the degree-w monomials, taken in
 * cell-local centred and scaled coordinates -- same span, better
 * conditioning) and wavelets spanning null(M).  Numerical rank: Householder
 * QR with column pivoting of M^T, |R_kk| > rank_rtol |R_00| (rank_rtol <= 0
 * selects 1e-10).  Coefficient layout of W v (N - p entries): level-major
 * from the finest level t down to 0, preorder cells within a level, V's
 * column order within a cell.  L v (p entries) are the root scaling
 * coefficients.  The basis keeps a reference to nothing: the tree may be
 * freed afterwards.  Root rank < p -> MLBLUP_ERANK; degree_w in [0, 16]. */
int mlblup_build_multilevel_basis(mlblup_tree t, int32_t degree_w, double rank_rtol, mlblup_basis* out);
/* p = binomial(d + w, w); levels = t + 1; device_bytes = size of the device
 * image mlblup_basis_upload writes. */
int mlblup_basis_info(mlblup_basis b, int32_t* p, int32_t* levels, int64_t* n_minus_p, int64_t* device_bytes);
/* Algorithmic bytes of one apply_W or apply_Wt (Sec. 6.2): every cell's
 * orthogonal block read once in the form the transform reads it: the
 * compact WY form I - Y T Y^T of the K = min(m, p) Householder reflectors
 * it is the product of (Y: K x m, T: K x K), 8 sum_cells (K m + K^2) (cells
 * of more than 256 candidates: the dense block, 8 m^2), plus the N-vector
 * read and the N-vector written, 16 N.  The HBM-roofline unit of the
 * transform. */
int mlblup_basis_transform_bytes(mlblup_basis b, int64_t* bytes);
/* Number of wavelets at level q = 0..t (levels entries). */
int mlblup_basis_level_counts(mlblup_basis b, int64_t* counts_host);
/* Dense W ((N-p) x N) and L (p x N), row-major, columns in TREE order.  For
 * tests on small N (N^2 doubles); either pointer may be NULL. */
int mlblup_basis_dense(mlblup_basis b, double* W_host, double* L_host);
/* Copies the basis device image (per-cell orthogonal blocks, the schedule,
 * the points in tree order, trend data) into dev_buf (>= device_bytes,
 * caller-owned, must outlive every device use of the basis).  Required once
 * before any call below that takes a basis. */
int mlblup_basis_upload(mlblup_basis b, void* dev_buf, int64_t bytes, void* stream);
/* Device pointer of the tree-ordered points inside the uploaded image. */
int mlblup_basis_points_dev(mlblup_basis b, const double** pts_dev);
void mlblup_basis_free(mlblup_basis b);

/* Host evaluation of sigma2 phi(r) for n distances r_host[i] >= 0 into
 * phi_host (host pointers): the same arithmetic as the FP64 pair kernels for
 * a general nu (table of genu.h), the closed forms otherwise.  For checking
 * and plotting; the products run on the device. */
int mlblup_matern_host(const mlblup_matern* k, const double* r_host, int64_t n, double* phi_host);

/* ---- dense covariance product (Sec. 6.2, step (2) of the chain) ----------
 * y_i = sum_j sigma2 phi(|r_i - c_j|) x_j over all m x n pairs (rows_dev:
 * m x d, cols_dev: n x d, row-major float64), and/or dy = (rho dC/drho) x.
 * The same pointer for rows and cols is allowed (square product).  Sums
 * are deterministic (fixed order, no atomics).  m = 0 or n = 0 gives y = 0.
 * precision: one of MLBLUP_FP64 .. MLBLUP_MFMA_BF16X3.  work_dev: at least
 * mlblup_cov_workspace_bytes(m, n, d, precision, outputs). */
int mlblup_cov_workspace_bytes(int64_t m, int64_t n, int32_t d, int32_t precision, int32_t outputs, int64_t* bytes);
int mlblup_cov_matvec(const mlblup_matern* k, const double* rows_dev, int64_t m, const double* cols_dev, int64_t n,
                      int32_t d, int32_t precision, int32_t outputs, const double* x_dev, double* y_dev,
                      double* dy_dev, void* work_dev, int64_t work_bytes, void* stream);

/* The same product for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): no workspace
 * argument, no hipMalloc / hipFree / event creation.  The scratch is a
 * static array of MLBLUP_NOALLOC_SCRATCH_BYTES in the library's device code,
 * one per GPU, held until the process ends; its address on the current
 * device is looked up on the first call there.  A product whose
 * mlblup_cov_workspace_bytes exceeds that size returns MLBLUP_EINVAL
 * (square FP64 values: up to about 226,000 points; both outputs: 113,000).
 * All calls on one GPU share the array: calls that overlap in time on the
 * same GPU (other streams, other threads) race and must not be issued.
 * Results are bitwise those of mlblup_cov_matvec.  Profiling
 * (mlblup_profile_enable) does not record these calls. */
#define MLBLUP_NOALLOC_SCRATCH_BYTES (64ll << 20)
int mlblup_cov_matvec_noalloc(const mlblup_matern* k, const double* rows_dev, int64_t m, const double* cols_dev,
                              int64_t n, int32_t d, int32_t precision, int32_t outputs, const double* x_dev,
                              double* y_dev, double* dy_dev, void* stream);

/* ---- multilevel transform (operators W and W^T, Sec. 3.1 and Sec. 6.2) -----
 * apply_W:  vw = W v (N - p), vl = L v (p; NULL to skip).
 * apply_Wt: v = W^T vw + L^T vl (vl NULL = 0).
 * work_dev: at least mlblup_transform_workspace_bytes(b). */
int mlblup_transform_workspace_bytes(mlblup_basis b, int64_t* bytes);
int mlblup_apply_W(mlblup_basis b, const double* v_dev, double* vw_dev, double* vl_dev, void* work_dev,
                   int64_t work_bytes, void* stream);
int mlblup_apply_Wt(mlblup_basis b, const double* vw_dev, const double* vl_dev, double* v_dev, void* work_dev,
                    int64_t work_bytes, void* stream);

/* ---- solve, predict, gradient (Sec. 6.2 predictor; Sec. 5.2 eqs. Spatial:eqn2-3)
 * Workspace for every call below: mlblup_solve_workspace_bytes(b, opts,
 * m_targets) (m_targets = largest target count used with it, 0 if none). */
int mlblup_solve_workspace_bytes(mlblup_basis b, const mlblup_pcg_opts* opts, int64_t m_targets, int64_t* bytes);

/* The operator of the Krylov solve: out = C_W in = W C(theta) W^T in, the
 * three-step product of Sec. 6.2 (W^T, the dense covariance product, W) in
 * the arithmetic `precision` of the pair kernel; in_dev and out_dev hold
 * N - p values (coefficients of the rows of W) and must not overlap.
 * Asynchronous on `stream`; workspace as for the solve (m_targets = 0). */
int mlblup_cw_matvec(mlblup_basis b, const mlblup_matern* k, const double* in_dev, double* out_dev,
                     int32_t precision, void* work_dev, int64_t work_bytes, void* stream);

/* Solves C_W gamma_W = zw by PCG (initial guess: gw_dev on entry when
 * use_x0 != 0, else 0).  An all-zero right-hand side returns gamma_W = 0.
 * Returns MLBLUP_ENOCONV with the last iterate if rtol is not reached. */
int mlblup_pcg_solve(mlblup_basis b, const mlblup_matern* k, const double* zw_dev, double* gw_dev, int32_t use_x0,
                     const mlblup_pcg_opts* opts, void* work_dev, int64_t work_bytes, mlblup_pcg_info* info,
                     void* stream);

/* Full predictor: Z_W = W z, solve, gamma = W^T gamma_W, beta from the least
 * squares of eq. Spatial:eqn3, Zhat(t) = k(t)^T beta + sum_j phi(|t - x_j|)
 * gamma_j at m_t targets (tgt_dev: m_t x d row-major).  beta_host: p
 * coefficients of the raw-coordinate monomials in graded lexicographic
 * order (1, x1, .., xd, x1^2, x1 x2, ..).  gamma_dev (N, tree order) and
 * gamma_w_dev (N - p) receive the solution; interp_res_host (may be NULL)
 * receives |W (z - C gamma)|_2, which equals |Zhat(S) - z|_2.  The final
 * products run in FP64 unless predict_precision says otherwise.
 * warm_start != 0: gamma_w_dev holds an initial guess on entry (e.g. the
 * solution of an earlier pcg_solve of the same system); the solve then
 * starts from it (one FP64 residual product when it already meets rtol). */
int mlblup_blup_predict(mlblup_basis b, const mlblup_matern* k, const double* z_dev, const double* tgt_dev,
                        int64_t m_t, const mlblup_pcg_opts* opts, int32_t predict_precision, int32_t warm_start,
                        double* zhat_dev, double* beta_host, double* gamma_dev, double* gamma_w_dev,
                        double* interp_res_host, void* work_dev, int64_t work_bytes, mlblup_pcg_info* info,
                        void* stream);

/* Quadratic form and its log-rho derivative (data term of the multilevel
 * likelihood, Sec. 3): Q = z . gamma (= Z_W . gamma_W) and
 * dQ/dlog rho = -lambda^T (rho dC/drho) gamma, lambda = gamma when
 * lambda_dev is NULL (the adjoint of Q is gamma itself), else the W^T image
 * of an adjoint solve.  One pass of the rho-derivative pair kernel
 * (MLBLUP_DLOGRHO output only) over the pairs; Q is a plain dot product. */
int mlblup_blup_grad(mlblup_basis b, const mlblup_matern* k, const double* z_dev, const double* gamma_dev,
                     const double* lambda_dev, int32_t precision, double* Q_host, double* dQ_dlogrho_host,
                     void* work_dev, int64_t work_bytes, void* stream);

/* ---- accuracy under ill-conditioning (Sec. 8, Table numericalresults:table5) ----
 * The multilevel predictor with the covariance formed in double-double
 * arithmetic, for small N (N <= 4096 sites, m_t <= 4096 targets) and
 * nu = 1/2, 3/2, 5/2 or +inf.  Every entry of P C P^T (P = [W; L], the dense
 * multilevel basis of Sec. 3.1) and of K(targets, S) P^T is formed in
 * double-double (about 32 digits) from the FP64 coordinates and basis, so W's
 * vanishing moments cancel the kernel's low-degree Taylor terms without
 * rounding noise (for the flat Gaussians of the experiment the entries of
 * C_W lie some 25 orders of magnitude below those of C, beneath the rounding
 * of any FP64 product).  C_W gamma_W = W z is solved by CG in FP64 on the
 * rounded C_W from gamma_W = 0, stopping when |W z - C_W gamma_W| <= rtol |W z|,
 * after max_iter iterations, or at a breakdown p.q <= 0 (the last iterate is
 * kept and the call still returns MLBLUP_OK).  Then, in double-double,
 * L v = L z - (L C W^T) gamma_W, (L X) beta = L v (X the raw-coordinate
 * monomials, graded-lex, Sec. 2) and zhat = X(targets) beta + (K W^T) gamma_W
 * (Sec. 5.2 eqs. Spatial:eqn1-3).
 * z_dev: N values in tree order; tgt_dev: m_t x d targets; zhat_dev: m_t values;
 * beta_host: p values (or NULL); cw_dev: optional (N-p) x (N-p) row-major copy
 * of the rounded C_W (NULL to skip); info_host: 4 doubles, the CG iterations,
 * 1 if it stopped at a breakdown, the recurrence and the true relative
 * residual.  Workspace: mlblup_dd_workspace_bytes(b, m_t).  Synchronises. */
int mlblup_dd_workspace_bytes(mlblup_basis b, int64_t m_t, int64_t* bytes);
int mlblup_blup_predict_dd(mlblup_basis b, const mlblup_matern* k, const double* z_dev, const double* tgt_dev,
                           int64_t m_t, double rtol, int32_t max_iter, double* zhat_dev, double* beta_host,
                           double* cw_dev, double* info_host, void* work_dev, int64_t work_bytes, void* stream);

/* ---- estimator: multilevel log-likelihood (Sec. 5.1 reduced likelihoods; Sec. 6.1) ----
 * For the levels q >= level of W (rows [W_t; ...; W_level], the first
 * N~ rows of W, finest level first):
 *   l = -N~/2 log(2 pi) - 1/2 log det C^n_W - 1/2 (Z^n_W)^T (C^n_W)^-1 Z^n_W,
 * C^n_W = [W_t; ..; W_level] C [W_t; ..; W_level]^T, Z^n_W = [..] z.
 * C^n_W is formed densely on the device from the N x N covariance and two
 * batched multilevel analyses, then factorized by a blocked FP64 Cholesky
 * G G^T = C^n_W: log det = 2 sum log G_ii, the quadratic form = |G^-1 Z^n_W|^2.
 * Any kernel of mlblup_matern.
 * tau: the distance of the sparsification of Sec. 4.1.  tau = INFINITY gives
 * the exact C^n_W.  A finite tau >= 0 gives the sparsified C~^n_W and l~: the
 * block of two cells B_a (level i) and B_b (level j >= i) is kept when the
 * kd-tree search from B_a reaches B_b at depth j, entering the left side of a
 * split (axis k, threshold s) when min_{B_a} x_k - tau <= s and the right
 * side when max_{B_a} x_k + tau > s (B_a's bounding box widened by tau meets
 * that side); blocks of one level are kept when either search connects the
 * pair, and every other block is zero.  The zeros are applied to the dense
 * matrix (the factorization is not shortened by them).  C~^n_W need not be
 * positive definite for small tau: then MLBLUP_EBREAKDOWN.
 * z_dev: N data values in tree order.  level: 0 .. levels - 1 (level 0 takes
 * all of W, where Z^0_W^T (C_W)^-1 Z^0_W is the Q of mlblup_blup_grad).
 * work_dev: at least the bytes from mlblup_loglik_workspace_bytes, which also
 * returns N~ in rows (may be NULL); about 8 (N^2 + N~ N) bytes plus at most
 * N~^2 + 4 N~ for the sparsity pattern, so N of a few
 * 10^4.  out4_host = {l, log det, quadratic form, kept entries of the N~ x N~
 * matrix}.  Synchronises `stream`.  MLBLUP_EINVAL for tau < 0 or NaN, a level
 * outside the range or a short workspace; MLBLUP_EBREAKDOWN if a Cholesky
 * pivot is not positive (not numerically positive definite, e.g. duplicate
 * points or a small tau). */
int mlblup_loglik_workspace_bytes(mlblup_basis b, int32_t level, int64_t* bytes, int64_t* rows);
int mlblup_loglik(mlblup_basis b, const mlblup_matern* k, const double* z_dev, int32_t level, double tau,
                  double* out4_host, void* work_dev, int64_t work_bytes, void* stream);
/* ---- estimator with the sparse factorization (Sec. 4.1 kept blocks; Sec. 6.1) ----
 * The same l (or l~ for a finite tau) as mlblup_loglik, computed without any
 * N x N or N~ x N~ array: only the blocks of C~^n_W that the tree search
 * keeps (the rule of mlblup_loglik) are formed, each block of two cells
 * B_a, B_b as Psi_a^T C(B_a, B_b) Psi_b from the cells' wavelet vectors on
 * their points, and the matrix is factored by a block Cholesky over the
 * cells (one block row and column per cell with wavelets at levels >=
 * level; a minimum-degree order of the cell graph, the fill blocks that
 * order creates, left-looking updates scheduled by elimination-tree
 * height), with Z^n_W as a border row for the quadratic form.  The last
 * columns of the order, which the fill makes nearly full, form a dense
 * tail: from the position where that is estimated to pay, the block
 * columns before it update it and the dense blocked Cholesky of
 * mlblup_loglik factors it (at most 49,152 rows; the environment variable
 * MLBLUP_SPARSE_TAIL=none or =all forces no tail or an all-dense one, and
 * MLBLUP_SPARSE_TAIL_MAX=<rows> lowers the row limit of a chosen tail, for
 * tests and measurement).  Cost and storage follow the kept blocks and
 * their fill, so a small tau makes it cheap; tau = INFINITY factors the
 * whole C^n_W (use mlblup_loglik there).  Every cell may own at most 64 wavelets: leaves of
 * at most 64 points and a trend dimension p <= 64 (else MLBLUP_EINVAL).
 * The analysis (pattern, order, block structure, wavelet vectors) is built
 * on the host on the first call for a (level, tau) and kept with the basis
 * for the following calls with the same pair.
 * mlblup_loglik_sparse_workspace_bytes: *bytes of device workspace;
 * info8_host (may be NULL) = {N~, kept entries of C~^n_W, doubles of the
 * block factor (with its fill), block columns before the dense tail,
 * elimination-tree heights of those columns, their factorization flops,
 * rows of the dense tail, its flops}.  No device access.
 * mlblup_loglik_sparse: z_dev N data values in tree order; out4_host = {l,
 * log det, quadratic form, kept entries}.  Synchronises `stream`.
 * MLBLUP_EINVAL as for mlblup_loglik or for a cell with more than 64
 * wavelets; MLBLUP_EBREAKDOWN if a pivot is not positive. */
int mlblup_loglik_sparse_workspace_bytes(mlblup_basis b, int32_t level, double tau, int64_t* bytes,
                                         double* info8_host);
int mlblup_loglik_sparse(mlblup_basis b, const mlblup_matern* k, const double* z_dev, int32_t level, double tau,
                         double* out4_host, void* work_dev, int64_t work_bytes, void* stream);
/* mlblup_mle_rho and mlblup_mle_nu_rho with every evaluation of l~ by
 * mlblup_loglik_sparse (same arguments and outputs; the workspace is that of
 * mlblup_loglik_sparse_workspace_bytes for (level, tau); the analysis is built
 * once). */
int mlblup_mle_rho_sparse(mlblup_basis b, const mlblup_matern* k, const double* z_dev, int32_t level, double tau,
                          double rho_lo, double rho_hi, double log_rho_tol, double* out4_host, void* work_dev,
                          int64_t work_bytes, void* stream);
int mlblup_mle_nu_rho_sparse(mlblup_basis b, double sigma2, const double* z_dev, int32_t level, double tau,
                             double nu_lo, double nu_hi, double nu_tol, double rho_lo, double rho_hi,
                             double log_rho_tol, double* out5_host, void* work_dev, int64_t work_bytes, void* stream);
/* The pattern of C~^n_W for the given level and tau (Sec. 4.1 search, the
 * rule of mlblup_loglik), on the host: *nnz = kept entries; mask_host (may be
 * NULL) receives the N~ x N~ row-major 0/1 matrix in the row order of
 * mlblup_loglik (caller-allocated, N~^2 bytes).  No device access. */
int mlblup_sparsity_pattern(mlblup_basis b, int32_t level, double tau, int64_t* nnz, uint8_t* mask_host);
/* Maximum-likelihood rho of l (or l~ for finite tau) at the given level, nu
 * and sigma2 of k fixed (k->rho is ignored): golden-section search on log rho
 * over [rho_lo, rho_hi] until the bracket is below log_rho_tol, each step one
 * mlblup_loglik evaluation (same workspace; the pattern is built once).
 * out4_host = {rho_hat, l(rho_hat), number of evaluations, final bracket width
 * in log rho}.  A maximum on the boundary of the bracket is returned as found
 * there. */
int mlblup_mle_rho(mlblup_basis b, const mlblup_matern* k, const double* z_dev, int32_t level, double tau,
                   double rho_lo, double rho_hi, double log_rho_tol, double* out4_host, void* work_dev,
                   int64_t work_bytes, void* stream);
/* Maximum-likelihood (nu, rho) of l (or l~) at the given level, sigma2 fixed,
 * by the profile likelihood: golden-section search over nu in [nu_lo, nu_hi]
 * (0 < nu_lo < nu_hi <= 8) until the bracket is below nu_tol, each point the
 * rho maximum of mlblup_mle_rho on [rho_lo, rho_hi].  out5_host = {nu_hat,
 * rho_hat, l(nu_hat, rho_hat), number of l evaluations, final nu bracket}. */
int mlblup_mle_nu_rho(mlblup_basis b, double sigma2, const double* z_dev, int32_t level, double tau, double nu_lo,
                      double nu_hi, double nu_tol, double rho_lo, double rho_hi, double log_rho_tol,
                      double* out5_host, void* work_dev, int64_t work_bytes, void* stream);

/* ---- preconditioner (remark on P_W = diag(C_W), Sec. 5.2) -----------------------
 * Built without forming C_W: the leaf kernel blocks and, for each internal
 * cell, the Gram of its children's scaling vectors across the two children
 * are summed on the device (about N^2/2 pairs over all levels, kernel values
 * with FP32 sqrt/exp), then each cell's wavelet block B_v = Psi_v^T C Psi_v
 * is assembled bottom-up on the host through the cell's orthogonal block.
 * JACOBI keeps diag(B_v) (= diag(C_W)); BLOCK keeps every B_v (inverted by
 * Cholesky).  Needs an uploaded basis with p <= 32.  The kernel parameters
 * are fixed at build time: rebuild when rho changes.  work_dev: at least
 * mlblup_precond_workspace_bytes(b).  Synchronises `stream`. */
int mlblup_precond_workspace_bytes(mlblup_basis b, int64_t* bytes);
/* MLBLUP_PREC_COARSE: the wavelets of every level above the finest (the
 * last nc rows of W, from c0 on) form one block C_c = W_c C W_c^T,
 * formed densely on the device (the N x N covariance and two batched
 * analyses) and factored G G^T = C_c with G^-T and G^-1 kept, rounded to
 * FP32 (2 nc^2 floats in the device image; the rounded pair is still an exact
 * symmetric positive definite preconditioner); the apply is two row products
 * with them (FP64 sums) plus the cell blocks of the finer wavelets.  Workspace about 8 (N^2 + nc N)
 * bytes, so N of about 10^5 at most; needs three or more levels with the
 * finest holding at least half of the rows (EINVAL otherwise).  This query
 * gives the workspace of any kind. */
int mlblup_precond_workspace_bytes_kind(mlblup_basis b, int32_t kind, int64_t* bytes);
int mlblup_precond_build(mlblup_basis b, const mlblup_matern* k, int32_t kind, void* work_dev, int64_t work_bytes,
                         void* stream, mlblup_precond* out);
/* device_bytes: size of the device image; n_blocks: cells with wavelets;
 * block_entries: sum of squared block sizes. */
int mlblup_precond_info(mlblup_precond pc, int64_t* device_bytes, int64_t* n_blocks, int64_t* block_entries);
/* Copies the device image into dev_buf (caller-owned, 256-byte aligned,
 * must outlive every solve that uses it). */
int mlblup_precond_upload(mlblup_precond pc, void* dev_buf, int64_t bytes, void* stream);
/* Host copies for tests: blocks B_v (row-major, concatenated in coefficient
 * order), each block's first coefficient and size (any pointer may be NULL). */
int mlblup_precond_blocks(mlblup_precond pc, double* blocks_host, int64_t* w_off_host, int32_t* mw_host);
/* Coarse kind, for tests: c0, nc and G^-T of the coarse block (nc x nc
 * row-major, host, caller-allocated; may be NULL).  Other kinds: nc = 0. */
int mlblup_precond_coarse(mlblup_precond pc, int64_t* c0, int64_t* nc, double* y_host);
void mlblup_precond_free(mlblup_precond pc);

/* ---- instrumentation --------------------------------------------------------
 * When enabled, each pair-kernel launch is bracketed by HIP events on its
 * own stream.  mlblup_profile_read fills three arrays of MLBLUP_PROF_BUCKETS
 * entries indexed by precision * 4 + outputs (precision MLBLUP_FP64 ..
 * MLBLUP_MFMA_BF16X3, outputs 1..3): summed kernel time in ms, launch
 * count, logical pair count since the last read, then resets them.  Any
 * pointer may be NULL.  Event timestamps are read with
 * hipEventSynchronize, so the streams used must be live. */
#define MLBLUP_PROF_BUCKETS 16
int mlblup_profile_enable(int32_t on);
int mlblup_profile_read(double* pair_ms, int64_t* launches, double* pairs);

#ifdef __cplusplus
}
#endif
#endif /* MLBLUP_H */
