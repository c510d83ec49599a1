/*
 * fkf.h - C ABI of the MI355X fast random-walk Kalman filter library (libfkf.so).
 *
 * The library implements the fast Kalman filter for the random-walk forecast
 * model of Saibaba, Miller & Kitanidis ("Fast Kalman filter using hierarchical
 * matrices and a low-rank perturbative approach"):
 *
 *   s_{k} = s_{k-1} + w_k,  w_k ~ N(0, Gamma)        (Section 2.1, F_k = I)
 *   y_k   = H_k s_k + v_k,  v_k ~ N(0, R_k)
 *
 * with the posterior covariance carried as Sigma_{k|k} = alpha_k Gamma - W D W^T
 * (Section 2.3, eq. sigmakk) and Gamma, a Matern covariance (eq. maternfamily),
 * held as a hierarchical matrix (Section 2.2.1).
 *
 * Conventions shared by every entry point
 *   - Every function is extern "C", never throws and never exits.  It returns
 *     FKF_OK or a negative fkf_status; fkf_last_error() then describes the
 *     failure (thread-local string, valid until the next failing call).
 *   - Arrays named *_host are host memory, read during the call and copied.
 *     Arrays named *_dev are device memory on the current HIP device, owned by
 *     the caller and accessed in stream order on `stream` (a hipStream_t passed
 *     as void*; NULL means the default stream).  All floating-point boundary
 *     buffers are float64.
 *   - Multi-column arrays are column-major with an explicit leading dimension.
 *   - Handles own all device memory they allocate; *_destroy frees it (after
 *     synchronising the device).  A handle is used by one thread at a time,
 *     and the device work of calls on one handle (which share its workspace)
 *     must not overlap: queue them on one stream, or synchronise between
 *     streams.
 *   - Argument errors are reported synchronously.  Numeric failures detected
 *     on the device (non-finite data, a non-positive-definite Gram matrix) are
 *     latched in the filter and reported by fkf_filter_status() and by the next
 *     fkf_filter_step(); a filter that has failed refuses further steps.
 *   - Points are given in the caller's order and every vector of length N
 *     (state, variance, draws) uses that order.
 */
#ifndef FKF_H
#define FKF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FKF_OK = 0,
  FKF_E_ARG = -1,          /* invalid argument (null, size, mismatch) */
  FKF_E_NOMEM = -2,        /* device allocation failed */
  FKF_E_HIP = -3,          /* a HIP runtime call failed */
  FKF_E_NOT_SPD = -4,      /* a matrix that must be positive definite is not */
  FKF_E_RANK = -5,         /* the low-rank term would exceed max_rank */
  FKF_E_NONFINITE = -6,    /* NaN/Inf met in data or state */
  FKF_E_ORDER = -7,        /* call out of order (e.g. step after a failure) */
  FKF_E_UNSUPPORTED = -8   /* valid request that this library does not support */
} fkf_status;

/* Matern smoothness nu = 1/2, 3/2, 5/2: the half-integer cases whose Bessel
 * form (eq. maternfamily) reduces to an exponential times a polynomial.
 * The *_DLENGTH kinds are the derivatives d/d length of those kernels,
 * (variance / length) (-t C'(t)) with t = c r / length: operators for
 * likelihood gradients (fkf_filter_track_length).  They are symmetric but not
 * positive definite, have zero diagonal, and cannot be a filter's
 * covariance. */
typedef enum {
  FKF_MATERN_12 = 0,
  FKF_MATERN_32 = 1,
  FKF_MATERN_52 = 2,
  FKF_MATERN_12_DLENGTH = 3,
  FKF_MATERN_32_DLENGTH = 4,
  FKF_MATERN_52_DLENGTH = 5
} fkf_kernel;

/* FKF_FP64: every H-matrix entry and every filter array in FP64.
 * FKF_MIXED: near-field blocks stored in FP32 (half the HBM bytes of the
 * dominant stream), far-field kernel entries evaluated in FP32, and the
 * constant-H basis streamed every step stored in FP32; all sums are
 * accumulated in FP64, and the projected eigenproblem, the innovation
 * Cholesky and the Gamma^-1-orthogonalisation stay in FP64. */
typedef enum { FKF_FP64 = 0, FKF_MIXED = 1 } fkf_precision;

/* Gamma[i,j] = variance * C_nu(|x_i - x_j| / length).  The paper's scaling
 * factor alpha of eq. maternfamily is 1/length; the variance multiplies it. */
typedef struct {
  uint32_t struct_size;   /* sizeof(fkf_kernel_params) */
  int32_t kind;           /* fkf_kernel */
  double variance;        /* theta > 0 */
  double length;          /* ell > 0 */
} fkf_kernel_params;

/* Hierarchical-matrix parameters (Section 2.2.1).  Clusters are built by
 * bisecting the longest side of each cluster's bounding box until at most
 * leaf_size points remain; (s, t) is admissible when
 * max(diam s, diam t) <= eta * dist(s, t).  Admissible blocks are
 * U_s K(xi_s, xi_t) U_t^T with tensor Chebyshev interpolation at p nodes per
 * dimension.  With block_tol > 0, p is raised per tree level (up to
 * cheb_order_max) until the sampled relative Frobenius error of the closest
 * admissible block of that level is <= block_tol (the paper chooses block
 * ranks by a relative Frobenius tolerance, Section 4.1.2); with
 * block_tol <= 0, p = cheb_order everywhere. */
typedef struct {
  uint32_t struct_size;   /* sizeof(fkf_hmat_params) */
  int32_t leaf_size;      /* 1..64 */
  int32_t cheb_order;     /* minimum p, 2..16 */
  int32_t cheb_order_max; /* maximum p when block_tol > 0 (>= cheb_order, <= 16) */
  double eta;             /* admissibility parameter, > 0 */
  double block_tol;       /* per-level block tolerance, or <= 0 */
  int32_t precision;      /* fkf_precision */
  int32_t far_eval;       /* 0: store the coupling matrices K(xi_s, xi_t) at build when they
                             take at most 8 GiB (faster one-column products); 1: evaluate
                             them in every product (no coupling storage) */
  int64_t workspace_bytes; /* bound on the workspaces of a several-column product
                              (gathered columns, coefficient vectors, upward partials,
                              all proportional to the number of columns); products with
                              more columns are applied in column blocks that fit.
                              0: 16 GiB */
} fkf_hmat_params;

/* Generalized eigensolver of the constant-H basis (Section 2.2.2):
 * FKF_GEP_EXACT: Rayleigh-Ritz on range(Gamma H^T) (exact: P = Gamma H^T,
 *   A = R^-1/2 H P R^-1/2 = W_e Lambda W_e^T in FP64, all n_m modes);
 * FKF_GEP_RANDOMIZED: the randomized algorithm of Appendix B with a Gaussian
 *   sketch Omega of k + p columns drawn on the device from `seed`
 *   (fkf_gaussian_sketch): Ybar = H^T R^-1 H Omega, a Gamma-orthonormal basis
 *   Qhat of range(Ybar) (two Gram eigen-decompositions in the Gamma inner
 *   product), Q = Gamma Qhat, T = (H Q)^T R^-1 (H Q) = S Lambda S^T, and the k
 *   largest modes U = Q S.  With k + p >= n_m the sketch spans range(H^T) and
 *   the modes are the exact ones; with fewer the filter assimilates what the
 *   k modes keep of each observation (H^T R^-1 H ~ Gamma^-1 U Lambda U^T
 *   Gamma^-1: the whitened data Lambda^-1/2 U^T H^T R^-1 y).  The steps of
 *   Section 2.4 (a new operator) need P for their gain anyway and always take
 *   the exact eigenpairs. */
enum { FKF_GEP_EXACT = 0, FKF_GEP_RANDOMIZED = 1 };

typedef struct {
  uint32_t struct_size;   /* sizeof(fkf_filter_params); the first three fields alone
                             (struct_size 16) are accepted, with the defaults below */
  int32_t max_rank;       /* capacity of the low-rank term W (>= n_m) */
  double rank_rtol;       /* relative truncation tolerance for W (Algorithm 5) */
  int32_t gep_mode;       /* FKF_GEP_EXACT (default) or FKF_GEP_RANDOMIZED */
  int32_t gep_rank;       /* k: modes kept by the randomized eigensolver (<= 0: n_m) */
  int32_t oversample;     /* p: extra sketch columns (< 0: 20, the appendix's choice) */
  int32_t reserved;       /* must be 0 */
  uint64_t seed;          /* sketch stream of the randomized eigensolver */
} fkf_filter_params;

/* Statistics of a built covariance operator. */
typedef struct {
  int64_t n;                 /* number of points */
  int32_t dim;               /* spatial dimension */
  int32_t n_leaves;
  int32_t n_levels;          /* tree depth + 1 */
  int64_t n_near_blocks;     /* stored near-field blocks (symmetric half) */
  int64_t n_near_pairs;      /* ordered near-field leaf pairs */
  int64_t n_far_pairs;       /* ordered admissible pairs */
  int64_t near_bytes;        /* bytes of stored near-field entries */
  int64_t far_coef_per_rhs;  /* sum over far clusters of p^dim */
  int32_t cheb_p[32];        /* Chebyshev nodes per dimension at each level */
  int64_t covered_entries;   /* sum of |s|*|t| over all blocks (= n*n for a partition) */
  int64_t far_interp_entries; /* sum over far clusters c of |c| * p_c^dim: interpolation-basis
                                  entries one upward (or downward) pass touches per column */
  int64_t far_bytes;         /* bytes of the stored coupling matrices K(xi_t, xi_s), one per
                                distinct geometry of an ordered admissible pair (s, t)
                                (pairs whose node counts, half-widths and centre offset
                                agree to 2^-40 of the extent share one); 0 when they are
                                evaluated on the fly (kept only up to 8 GiB) */
  int64_t far_pair_entries;  /* entries of the coupling matrices of all unordered admissible
                                pairs (the work of one coupling pass per column) */
  int64_t coupling_groups;   /* one-column product with stored couplings: groups of far
                                clusters that couple through the same sequence of stored
                                matrices (0 when the per-cluster kernel is used) */
  int64_t coupling_items;    /* work items of the grouped one-column couplings */
} fkf_cov_info_t;

typedef struct fkf_cov fkf_cov;
typedef struct fkf_obs fkf_obs;
typedef struct fkf_filter fkf_filter;

/* ---------------------------------------------------------------- Gamma --- */

/* Build Gamma_sys as an H-matrix over n points of dimension d (2 or 3).
 * pts_host: n x d row-major coordinates.  Assembles the near-field blocks on
 * the device (Section 2.2.1; the paper's construction cost is O(k^2 N),
 * Section 4.1.2).  Besides the near tiles (near_bytes of fkf_cov_info_t) the
 * operator keeps the tiles of all n_near_pairs ordered near pairs once more,
 * in the operand order of the several-column product (64 x 64 entries each,
 * FP64, or FP32 in the mixed mode).  On success *out owns all device memory
 * of the operator. */
fkf_status fkf_cov_build(const double *pts_host, int64_t n, int32_t d,
                         const fkf_kernel_params *kernel,
                         const fkf_hmat_params *hmat, void *stream,
                         fkf_cov **out);

/* Y = Gamma X for X_dev (n x nrhs, leading dimension ldx >= n) into Y_dev
 * (n x nrhs, ldy >= n).  X and Y must not overlap.  This is the matrix-vector
 * product the paper names as the dominant cost (Section 2.5): the cross
 * covariance Gamma H^T and the products inside the eigensolver.  nrhs = 0 is
 * a no-op.  Uses a workspace held by the handle (grown on demand). */
fkf_status fkf_cov_apply(fkf_cov *cov, const double *X_dev, int64_t ldx,
                         int32_t nrhs, double *Y_dev, int64_t ldy, void *stream);

/* The product of fkf_cov_apply (same arguments, same kernels, same result)
 * for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  It calls
 * no hipMalloc/hipFree: the workspace lives in a fixed 64 MiB array of device
 * memory per GPU that the library holds from its load until the process
 * ends, and the columns are applied in blocks whose workspace fits it
 * (one column at a time when two do not fit).  FKF_E_ARG when even the
 * one-column workspace of the operator (8 bytes per point plus the near-field
 * partials and far-field vectors, about 6 MiB at N = 65536) exceeds it.  All
 * calls on one GPU share that array: calls whose device work overlaps (on
 * different streams, or from different threads) race and give wrong
 * results, so serialise them. */
fkf_status fkf_cov_apply_noalloc(fkf_cov *cov, const double *X_dev, int64_t ldx,
                                 int32_t nrhs, double *Y_dev, int64_t ldy, void *stream);

fkf_status fkf_cov_info(const fkf_cov *cov, fkf_cov_info_t *info);

/* Host-only planning: builds the cluster tree, the block partition and the
 * per-level Chebyshev orders exactly as fkf_cov_build does and reports them,
 * without touching the GPU. */
fkf_status fkf_cov_plan(const double *pts_host, int64_t n, int32_t d,
                        const fkf_kernel_params *kernel, const fkf_hmat_params *hmat,
                        fkf_cov_info_t *info);

/* Tree-order permutation (perm_host[i] = caller index of tree position i). */
fkf_status fkf_cov_perm(const fkf_cov *cov, int64_t *perm_host);

void fkf_cov_destroy(fkf_cov *cov);

/* ----------------------------------------------------------- observations --- */

/* Measurement operator H (n_m x n) from host CSR arrays (rowptr has n_m+1
 * entries, col in [0, n)), plus the diagonal of the noise covariance R
 * (noise_var_host, n_m entries, each > 0).  The stored rows are sorted by
 * column with repeated columns summed (fkf_obs_shape and fkf_obs_get_csr
 * report that form; both constructors store it). */
fkf_status fkf_obs_create_csr(int32_t n_m, int64_t n, const int64_t *rowptr_host,
                              const int32_t *col_host, const double *val_host,
                              const double *noise_var_host, void *stream,
                              fkf_obs **out);

/* Straight-ray travel-time operator on a regular grid of the unit square/cube
 * (Section 4.1, eq. lineartomography): H[m, c] is the length of the segment
 * src_m -> rcv_m inside cell c.  grid_host holds d cell counts; cell
 * (i, j[, k]) has flat index i + nx*(j + ny*k).  A ray is cut at every grid
 * line/plane crossing; a piece lying exactly on an interior grid line/plane is
 * shared equally by the cells on both sides.  src_host, rcv_host: n_m x d
 * row-major. */
fkf_status fkf_obs_create_rays(int32_t d, const int32_t *grid_host, int32_t n_m,
                               const double *src_host, const double *rcv_host,
                               const double *noise_var_host, void *stream,
                               fkf_obs **out);

/* Host-only form of the ray operator above (no GPU): writes rowptr_host
 * (n_m + 1 entries) and *nnz; when col_host/val_host are non-NULL they must
 * hold `capacity` entries and receive the CSR columns/values (FKF_E_ARG when
 * capacity < nnz). */
fkf_status fkf_rays_host(int32_t d, const int32_t *grid_host, int32_t n_m,
                         const double *src_host, const double *rcv_host,
                         int64_t *rowptr_host, int64_t *nnz, int32_t *col_host,
                         double *val_host, int64_t capacity);

/* Sizes of H; nnz may be NULL. */
fkf_status fkf_obs_shape(const fkf_obs *obs, int32_t *n_m, int64_t *n, int64_t *nnz);

/* Copy H out as CSR to host arrays sized from fkf_obs_shape. */
fkf_status fkf_obs_get_csr(const fkf_obs *obs, int64_t *rowptr_host,
                           int32_t *col_host, double *val_host);

/* y_dev (n_m) = H x_dev (n). */
fkf_status fkf_obs_apply(const fkf_obs *obs, const double *x_dev, double *y_dev,
                         void *stream);

/* P_dev (n x n_m, leading dimension ldp >= n) = Gamma H^T, the cross
 * covariance whose range carries the Rayleigh-Ritz step of the generalized
 * eigenproblem (Section 2.2.2; in the offline stage of Section 4.1.2 H is
 * sparse and the products with Gamma dominate).  The moments of the far
 * clusters are summed over the nonzeros of H; an operator without far field,
 * or an H with a row of more than 2048 entries, takes fkf_cov_apply of the
 * dense H^T instead.  Either way the result equals fkf_cov_apply of the dense
 * H^T up to rounding order.  cov and obs must have the same n (FKF_E_ARG
 * otherwise); P must not overlap the operator's memory.  Allocates a dense
 * H^T (8 n n_m bytes) for the call and synchronises the stream before
 * returning. */
fkf_status fkf_obs_cross_cov(fkf_cov *cov, const fkf_obs *obs, double *P_dev, int64_t ldp,
                             void *stream);

void fkf_obs_destroy(fkf_obs *obs);

/* ----------------------------------------------------------------- filter --- */

/* Create a filter with s_{0|0} = s0_dev (NULL: zero) and
 * Sigma_{0|0} = alpha0 * Gamma, alpha0 >= 0 (Section 2.3; the experiments use
 * s_0 = Sigma_0 = 0, i.e. alpha0 = 0).  params may be NULL for defaults. */
fkf_status fkf_filter_create(fkf_cov *cov, const double *s0_dev, double alpha0,
                             const fkf_filter_params *params, void *stream,
                             fkf_filter **out);

/* Return f to the state fkf_filter_create gives (s_{0|0} = s0_dev or zero,
 * Sigma_{0|0} = alpha0 Gamma, no step taken, no basis, no latched failure,
 * log-likelihood zero; a length derivative set by fkf_filter_track_length
 * stays tracked), keeping every device buffer the filter has allocated so
 * that running it again over new data allocates nothing while the operators
 * keep their sizes.  Synchronises the stream. */
fkf_status fkf_filter_reset(fkf_filter *f, const double *s0_dev, double alpha0, void *stream);

/* One predict + update with observations y_dev (n_m values) of operator obs.
 * Prediction: alpha <- alpha + 1, estimate unchanged (F = I).  Update:
 * while the filter's low-rank basis is that of obs (the first step, and every
 * later step with the same obs), the constant-H update of Algorithms 2/3
 * using the generalized eigenpairs of obs (computed once, Section 2.2.2);
 * a step with a different obs after that uses the update of Section 2.4. */
fkf_status fkf_filter_step(fkf_filter *f, const fkf_obs *obs, const double *y_dev,
                           void *stream);

/* Innovation log-likelihood of the steps taken so far,
 *   ll = sum_k -(nu_k^T S_k^-1 nu_k + log det S_k + n_m log 2 pi) / 2,
 * with innovation nu_k = y_k - H_k s_{k|k-1} (for the extended filter,
 * y_k - h(s_{k|k-1})) and S_k = H_k Sigma_{k|k-1} H_k^T + R_k: the Gaussian
 * likelihood of y_1..y_k under the model of Section 2.1 in prediction-error
 * form (a quantity the paper does not compute; it is what parameter
 * estimation of theta, length and the noise level differentiates).  *ll
 * receives it (0 before the first step).  dll_dlog_theta, dll_dlog_length
 * and dll_dlog_noise (each may be NULL) receive its exact derivatives with
 * respect to log theta (Gamma scaled as a whole), log length (the Matern
 * length; requires fkf_filter_track_length, else FKF_E_ORDER) and
 * log sigma^2 (every R_k scaled as a whole).  They are carried in forward
 * mode through the recursion of the constant-H filter in the whitened
 * eigenbasis of its operator, in which the data-space covariance is diagonal:
 * theta and sigma^2 keep it diagonal (O(n_m) per step), the length tangent
 * is a full n_m x n_m matrix (O(n_m^2) per step).  Derivatives are available
 * while every step so far was a constant-H step (FKF_E_UNSUPPORTED after a
 * step of Section 2.4 or a second extended-filter step).  Synchronises
 * `stream`. */
fkf_status fkf_filter_loglik(const fkf_filter *f, double *ll, double *dll_dlog_theta,
                             double *dll_dlog_length, double *dll_dlog_noise, void *stream);

/* Track d ll / d log length in f (see fkf_filter_loglik): dcov is the
 * operator dGamma/d length, built by fkf_cov_build on the same points with
 * the same variance, length and H-matrix parameters and the kind
 * FKF_MATERN_*_DLENGTH of f's kernel (only its kind, size and length are
 * checked; FKF_E_ARG).  Must be called before the first step (FKF_E_ORDER).
 * The basis build then costs one more n_m-column product with dcov and two
 * N x n_m x n_m products; each constant-H step one O(n_m^2) update.  dcov is
 * borrowed: it must outlive f's steps and log-likelihood queries. */
fkf_status fkf_filter_track_length(fkf_filter *f, fkf_cov *dcov, void *stream);

/* One step of the extended Kalman filter for the Box-Cox observation model
 * (numerical experiments, Extended Kalman Filter; Algorithm 4).  The filter's
 * state is the transformed field x; the physical field is
 * s = g(x) = ((x + a)/a)^a with a = bc_alpha, the inverse of the Box-Cox
 * transform x = a (s^(1/a) - 1) (eq. nonlinear), and y_dev (n_m values) are
 * measurements y = H g(x) + v of obs's operator H and noise.  Prediction as
 * in fkf_filter_step.  The update linearises h(x) = H g(x) about the
 * predicted estimate, H_k = H diag(g'(x)) with g'(x) = ((x + a)/a)^(a-1), and
 * is the update of fkf_filter_step for H_k with the innovation y - H g(x)
 * (one linearisation per step).  Below the transform's domain (x < -a) the
 * base (x + a)/a is taken as 0: g = 0 and g' is its one-sided limit at the
 * edge (1 for a = 1, else 0).  H_k changes from step to step, so the first
 * step builds the constant-H basis of H_0 and every later step takes the
 * update of Section 2.4; fkf_filter_params.rank_rtol truncates the low-rank
 * term there (the paper uses 1e-5).  bc_alpha must be finite and > 0
 * (FKF_E_ARG).  fkf_filter_mean and fkf_filter_variance report x and its
 * variances.  The linearised operator and data are held by the filter (n_m
 * + nnz doubles, reused while obs is the same). */
fkf_status fkf_filter_step_boxcox(fkf_filter *f, const fkf_obs *obs, double bc_alpha,
                                  const double *y_dev, void *stream);

/* One step of count independent filters: the same as calling
 * fkf_filter_step(filters[i], obs[i], y[i]) for i = 0..count-1 in order,
 * except that the projected eigenproblems (Section 2.2.2) of all filters that
 * build their constant-H basis in this step are solved together, as one
 * batch of eigenproblems in one sequence of launches (the many-filter form of
 * the method: independent filters of uneven size share the latency-bound
 * eigensolver rounds).  filters, obs and y are host arrays of count handles /
 * device pointers (each y[i] of length obs[i]'s n_m); a filter may appear
 * only once.  The argument and state checks of fkf_filter_step are made for
 * every filter before any work is queued, so such an error leaves every
 * filter unchanged. */
fkf_status fkf_filter_step_many(fkf_filter *const *filters, const fkf_obs *const *obs,
                                const double *const *y, int32_t count, void *stream);

/* Synchronise `stream` and return the latched device-side status. */
fkf_status fkf_filter_status(fkf_filter *f, void *stream);

/* s_dev (n) = current estimate s_{k|k}. */
fkf_status fkf_filter_mean(const fkf_filter *f, double *s_dev, void *stream);

/* var_dev (n) = diag Sigma_{k|k} = alpha_k diag Gamma - diag(W D W^T)
 * (Section 3.1). */
fkf_status fkf_filter_variance(const fkf_filter *f, double *var_dev, void *stream);

/* Conditional realizations (Section 3.3):
 * out[:, j] = s_{k|k} + alpha^{1/2} (g_j - W Sigma_- W^T Gamma^{-1} g_j), with
 * Sigma_- = I - (I - D/alpha)^{1/2}.  g_dev holds ns unconditional draws
 * g ~ N(0, Gamma) (n x ns, leading dimension ldg); out_dev is n x ns (ldo). */
fkf_status fkf_filter_realize(const fkf_filter *f, const double *g_dev, int32_t ns,
                              int64_t ldg, double *out_dev, int64_t ldo, void *stream);

/* The Gaussian numbers of the randomized eigensolver's sketch (Appendix B):
 * out_dev[e] for e = 0..count-1 is number e of stream `seed` (element (i, j)
 * of the n x (k + p) column-major sketch is number i + n j).  Counter-based:
 * Philox4x32-10 (Salmon et al., SC 2011) of the counter (e/2 mod 2^32,
 * e/2 div 2^32, 0, 0) under the key (seed mod 2^32, seed div 2^32); with
 * outputs x0..x3, u1 = ((x0 >> 6) 2^27 + (x1 >> 5) + 1/2) 2^-53 and u2 from
 * x2, x3 likewise, the Box-Muller pair sqrt(-2 ln u1) (cos, sin)(2 pi u2)
 * gives numbers e (cosine, e even) and e + 1 (sine). */
fkf_status fkf_gaussian_sketch(uint64_t seed, int64_t count, double *out_dev, void *stream);

/* Eigen-decomposition of a symmetric n x n FP64 matrix on the device: the
 * solver of the projected eigenproblem of the generalized eigenvalue
 * problem (Section 2.2.2, eq. geneigendecomposition) and of the small
 * symmetric problems of the low-rank updates (Section 2.4, Algorithm 5).
 * A (device, column-major, lda >= n; read only, both triangles are read and
 * must agree) -> w (device, n eigenvalues in descending order) and W
 * (device, n x n column-major, ldw >= n; column i the unit eigenvector of
 * w[i]; W must not overlap A).  Orders 3..1024 take Householder
 * tridiagonalization, divide and conquer and back-transformation; other
 * orders take two-sided block Jacobi (off-diagonal norm below
 * 1e-12 ||A||_F).  The workspace is allocated and freed inside the call,
 * which synchronises the stream before it returns.  FKF_E_ARG for n < 1,
 * lda < n, ldw < n or a null pointer; FKF_E_HIP when the workgroups of the
 * reduction could not all run at once (the outputs are then undefined). */
fkf_status fkf_sym_eig(const double *A, int64_t lda, int32_t n, double *w, double *W,
                       int64_t ldw, void *stream);

/* Step count k, alpha_k and the rank of the low-rank term (any may be NULL). */
fkf_status fkf_filter_info(const fkf_filter *f, int64_t *k, double *alpha,
                           int32_t *rank);

/* Constant-H basis: the generalized eigenvalues lambda (descending) and the
 * per-mode weights c = alpha - D of Sigma in the basis Gamma^{-1} U, copied to
 * host arrays of length `rank` (as returned by fkf_filter_info).  Returns
 * FKF_E_ORDER when the filter is not in the constant-H form. */
fkf_status fkf_filter_modes(const fkf_filter *f, double *lambda_host,
                            double *weight_host);

/* The low-rank term of Sigma_{k|k} = alpha_k Gamma - W D W^T (Section 2.3,
 * eq. sigmakk; Section 2.4 for the general form) with its dual
 * Wd = Gamma^-1 W, so that W^T Gamma^-1 W = Wd^T W = I: copies W and Wd
 * (n x r, caller order, leading dimensions ldw, ldwd >= n) and D (r values)
 * to device arrays with room for `capacity` columns (at least the rank of
 * fkf_filter_info, else FKF_E_ARG) and writes r to *rank (0 before the first
 * step).  In the constant-H form the columns are the generalized
 * eigenvectors U = U0 Lambda^-1/2 with lambda > 1e-13 lambda_max (the others
 * carry no weight, Gamma^-1-norm sqrt(lambda)), Wd = H^T R^-1/2 W_e
 * Lambda^-1/2 and D the per-mode weights of Algorithms 2 and 3; in the general form the
 * stored W, Wd and D.  Any of W_dev, Wd_dev, D_dev may be NULL.  A query for
 * tests and diagnostics: in the constant-H form it allocates a dense H^T
 * (8 n n_m bytes); it synchronises the stream. */
fkf_status fkf_filter_lowrank(const fkf_filter *f, double *W_dev, int64_t ldw, double *Wd_dev,
                              int64_t ldwd, double *D_dev, int32_t capacity, int32_t *rank,
                              void *stream);

void fkf_filter_destroy(fkf_filter *f);

/* -------------------------------------------------------------------- misc --- */

const char *fkf_last_error(void);

/* Tracing: when enabled (on != 0), the library records a HIP event pair on the
 * launch stream around each instrumented launch site (the round launches of
 * one eigensolver sweep share one pair, so no events separate those
 * back-to-back kernels); fkf_trace_query returns the number of recorded
 * launches of a site and their summed duration in milliseconds (synchronising
 * on the recorded events).  Enabling or disabling
 * synchronises the device and clears all records.  Site names are listed,
 * comma-separated, by fkf_trace_names (FKF_E_ARG when cap is too small). */
fkf_status fkf_trace_enable(int32_t on);
fkf_status fkf_trace_query(const char *name, int64_t *count, double *total_ms);
fkf_status fkf_trace_names(char *buf, int64_t cap);

/* Library version string. */
const char *fkf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FKF_H */
