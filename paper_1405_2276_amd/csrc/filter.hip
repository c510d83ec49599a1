// Measurement operators and the fast random-walk Kalman filter on the GPU.
//
// The filter keeps Sigma_{k|k} = alpha_k Gamma - W D W^T (Section 2.3,
// eq. sigmakk).  For a measurement operator H with noise R it uses the
// generalized eigenpairs of H^T R^-1 H x = lambda Gamma^-1 x (Section 2.2.2),
// obtained exactly by Rayleigh-Ritz on range(Gamma H^T):
//   P = Gamma H^T (H-matrix product), A = R^-1/2 (H P) R^-1/2 = W_e Lambda W_e^T,
//   U = P R^-1/2 W_e Lambda^-1/2,  Gamma^-1 U = H^T R^-1/2 W_e Lambda^-1/2,
// so that U^T Gamma^-1 U = I and H^T R^-1 H = Gamma^-1 U Lambda U^T Gamma^-1.
// Device state for the constant-H form (W = U): U0 = P R^-1/2 W_e (n x n_m),
// Ve = R^-1/2 W_e, lambda, and delta = D / lambda (finite as lambda -> 0).
//
// Constant-H step (Algorithms 2 and 3): alpha <- alpha + 1; with a = alpha - D
// per mode, S_k is diagonal in the eigenbasis with entries a lambda + 1, the
// gain applied to the innovation is U0 diag(a / (1 + a lambda)) Ve^T nu, and
// D <- D + a^2 lambda / (1 + a lambda) (the printed update
// D + ((a)^-1 Lambda^-1 + I)^-1 a), i.e. delta <- delta + a^2 / (1 + a lambda).
//
// General form (a step with an operator other than the basis', Section 2.4):
// Sigma = alpha Gamma - W D W^T with W^T Gamma^-1 W = I, stored with its dual
// Wd = Gamma^-1 W so that no product with Gamma^-1 is ever formed: every
// column the filter creates lies in range(Gamma H^T), whose dual is H^T Z.
// The step uses the gain F = Sigma_{k+1|k} H^T = alpha P - W D (H W)^T, the
// innovation covariance S = H F + R (FP64 Cholesky), and updates the
// covariance by adding the low-rank terms of Sigma^-1 with Algorithm 5
// (B = Gamma^-1 realised through the duals), then D = alpha^2 Dh / (1 + alpha Dh).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>

#include "kernels.h"
#include "linalg.h"
#include "trace.h"

struct fkf_obs {
  int n_m = 0;
  int64_t n = 0, nnz = 0;
  int64_t max_row = 0;     // entries in the longest row
  uint64_t gen = 0;
  std::vector<int64_t> rowptr_h;
  std::vector<int32_t> col_h;
  std::vector<double> val_h, noise_h;
  // rows of ray operators in Morton order of their endpoints (rays that cross
  // the same region close together; empty for a CSR operator): the order in
  // which the cross covariance takes them as columns, so that a cluster's
  // moments are nonzero in few 16-column blocks
  std::vector<int32_t> order_h;
  fkf::DevBuf<int32_t> order;
  fkf::DevBuf<int64_t> rowptr;
  fkf::DevBuf<int32_t> col;
  fkf::DevBuf<double> val, noise, inv_sqrt_noise;
  double ll_const = 0.0;   // -(sum log R + n_m log 2 pi) / 2
};

// Workspaces of a constant-H basis build (cross covariance, Gram matrices,
// the dense H^T where needed), kept by the filter so that a rebuild after
// fkf_filter_reset allocates nothing.
struct BasisWork {
  fkf::DevBuf<double> Ht, P, G, A, X;
};

struct fkf_filter {
  fkf_cov *cov = nullptr;
  BasisWork bw;
  int64_t n = 0, ldu = 0;
  double theta = 1.0;
  fkf_filter_params params{};
  int64_t k = 0;
  double alpha = 0.0;
  int mode = 0;            // 0: no low-rank term yet, 1: constant-H basis, 2: general
  uint64_t basis_gen = 0;
  int n_m = 0;             // data dimension of the basis' operator
  int nmode = 0;           // modes of the constant-H basis (columns of U0 and Ve)
  fkf_status failed = FKF_OK;
  fkf::DevBuf<double> s, U0, Ve, lam, delta, nu, zp, tmp, eta;
  bool mixed = false;              // mixed-precision covariance: U0 also kept in FP32
  fkf::DevBuf<float> U0f;          // FP32 copy of U0 streamed by the per-step GEMVs
  fkf::DevBuf<int64_t> b_rowptr;   // copy of the basis' measurement operator
  fkf::DevBuf<int32_t> b_col;
  fkf::DevBuf<double> b_val;
  fkf::DevBuf<int> err;
  int *err_host = nullptr;
  fkf::EigWork eig;
  // general form (mode 2): W, Wd = Gamma^-1 W (n x rg, ld ldu), D (rg)
  fkf::DevBuf<double> W, Wd, Dg;
  int rg = 0;
  // scratch reused across general steps
  fkf::DevBuf<double> gP, gHt, gG, gA, gWe, glam, gwork, gtmp;
  fkf::DevBuf<double> gdv, gll;    // state increment and log-density of a general step,
                                   // committed only when the whole step succeeds
  fkf::DevBuf<int> chol_flag;
  // innovation log-likelihood: per-mode terms and tangents of the constant-H
  // steps (llq), the sum over general steps (ll_gen, device), the whitening
  // constants of the constant-H steps (host), and whether a general step
  // has been taken (its log-likelihood has no tangents)
  fkf::DevBuf<double> llq, ll_gen;
  double ll_const = 0.0;
  bool ll_general = false;
  // length derivative (fkf_filter_track_length): dGamma/d ell, the tangent
  // operator Ad and the tangent covariance Cd in the whitened eigenbasis
  fkf_cov *dcov = nullptr;
  fkf::DevBuf<double> ll_Ad, ll_Cd;
  // extended filter (Box-Cox model): operator H_k linearised about the
  // estimate (same sparsity as the source operator, whose generation is
  // lin_src) and the data of the equivalent linear step
  std::unique_ptr<fkf_obs> lin;
  uint64_t lin_src = 0;
  fkf::DevBuf<double> ytil;
  ~fkf_filter() {
    if (err_host) (void)hipHostFree(err_host);
  }
};

namespace fkf {

// implemented in hmat.hip
double cov_variance(const fkf_cov *cov);
int64_t cov_n(const fkf_cov *cov);
bool cov_mixed(const fkf_cov *cov);
int cov_kind(const fkf_cov *cov);
double cov_length(const fkf_cov *cov);
// Gamma H^T from the rows of the sparse H (CSR, device): false, with nothing
// queued, where that form does not apply.  order (device, n_m, or null): the
// rows in the order in which they are taken as columns of the product (the
// result is in row order either way).
bool cov_apply_sparse_rows(fkf_cov *cov, int n_m, const int64_t *rowptr, const int32_t *col,
                           const double *val, int64_t nnz, int64_t max_row, const int32_t *order,
                           double *Y, int64_t ldy, hipStream_t st);

static std::atomic<uint64_t> g_obs_gen{1};


// ------------------------------------------------------------- kernels ---
__global__ void __launch_bounds__(256) k_innov(const int64_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col,
                                               const double *__restrict__ val, int n_m,
                                               const double *__restrict__ s,
                                               const double *__restrict__ y,
                                               double *__restrict__ nu, int *err) {
  int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= n_m) return;
  int l = threadIdx.x & 63;
  double acc = 0;
  for (int64_t e = rowptr[m] + l; e < rowptr[m + 1]; e += 64) acc = fma(val[e], s[col[e]], acc);
  acc = wave_sum(acc);
  if (l == 0) {
    double v = y[m] - acc;
    if (!isfinite(v)) atomicExch(err, (int)FKF_E_NONFINITE);
    nu[m] = v;
  }
}

// Innovation log-likelihood of the constant-H filter, mode by mode.  In the
// whitened eigenbasis (u = Ve^T y) the data-space filter decouples into n_m
// scalar random walks: mode j has predicted variance p- = (alpha - D_j)
// lambda_j, innovation variance S = p- + 1 and innovation z_j, and
// contributes -(z^2/S + log S)/2 per step (the whitening's -(sum log R +
// n_m log 2 pi)/2 is added on the host).  Scaling Gamma by A and R by s
// changes only the scalar recursions (p- = p + A lambda, S = p- + s), so the
// derivatives with respect to log theta and log sigma^2 at A = s = 1 follow
// by carrying the tangents of the mode's posterior variance p and mean m
// (forward mode).  Per mode: q = [dp/dA, dp/ds, dm/dA, dm/ds, ll, dll/dA,
// dll/ds, p- and z of the latest step, dll/d ell (row sums, see
// k_loglik_length_step), dm/d ell, unused].
constexpr int kLLStride = 12;

__device__ __forceinline__ void loglik_mode_step(double *__restrict__ q, double pm, double lj,
                                                 double z) {
  const double S = pm + 1.0;
  const double iS = 1.0 / S;
  const double pmA = q[0] + lj, pmS = q[1];
  const double SA = pmA, SS = pmS + 1.0;
  const double eA = -q[2], eS = -q[3];
  const double e2 = z * z * iS;
  q[4] += -0.5 * (e2 + log(S));
  q[5] += -0.5 * ((2.0 * z * eA - e2 * SA + SA) * iS);
  q[6] += -0.5 * ((2.0 * z * eS - e2 * SS + SS) * iS);
  const double G = pm * iS;                       // gain of the mode's mean
  const double GA = (pmA - G * SA) * iS, GS = (pmS - G * SS) * iS;
  q[2] += GA * z + G * eA;
  q[3] += GS * z + G * eS;
  q[0] = GA;                                      // posterior p = s p- / S
  q[1] = G + GS;
  q[7] = pm;
  q[8] = z;
}

// Derivative of the log-likelihood with respect to the length scale.  In
// the whitened eigenbasis of the reference operator the data-space
// covariance C of the filter is diagonal, but its tangent Cd under
// Gamma -> Gamma + d ell dGamma/d ell is a full matrix: it starts at
// alpha_0 Ad (Ad = Ve^T H (dGamma/d ell) H^T Ve) and per step
//   Cd- = Cd + Ad,  S = diag(p- + 1),  g = p- / S,
//   dll += -(tr(S^-1 Cd-) - 2 z^T S^-1 dm - (S^-1 z)^T Cd- (S^-1 z)) / 2,
//   dm <- dm + (1 - g) o (Cd- S^-1 z) - g o dm,   Cd <- Cd- o (1 - g)(1 - g)^T
// (the tangents of the innovation terms, of the gain update of the mean and
// of C = C- - C- S^-1 C-), O(n_m^2) per step.  One wavefront per row i; the
// symmetric Cd is stored whole and wavefront i reads and writes column i.
__global__ void __launch_bounds__(256) k_loglik_length_step(int n_m, const double *__restrict__ Ad,
                                                            double *__restrict__ Cd,
                                                            double *__restrict__ q) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n_m) return;
  const int l = threadIdx.x & 63;
  double *qi = q + (int64_t)kLLStride * i;
  const double si = 1.0 + qi[7], gi = qi[7] / si, zi = qi[8];
  double r = 0.0, dii = 0.0;
  double *col = Cd + (int64_t)n_m * i;
  const double *acol = Ad + (int64_t)n_m * i;
  for (int j = l; j < n_m; j += 64) {
    const double *qj = q + (int64_t)kLLStride * j;
    const double sj = 1.0 + qj[7], gj = qj[7] / sj;
    const double cm = col[j] + acol[j];
    r = fma(cm, qj[8] / sj, r);
    if (j == i) dii = cm;
    col[j] = cm * (1.0 - gi) * (1.0 - gj);
  }
  r = wave_sum(r);
  dii = wave_sum(dii);
  if (l == 0) {
    const double dm = qi[10];
    qi[9] += -0.5 * (dii / si - 2.0 * zi * dm / si - zi / si * r);
    qi[10] = dm + (1.0 - gi) * r - gi * dm;
  }
}

// Tangent state at the basis build: p = alpha lambda_j (so dp/dA = p), the
// rest zero.
__global__ void k_loglik_init(double *__restrict__ q, const double *__restrict__ lam, int n_m,
                              double alpha) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_m) return;
  double *r = q + (int64_t)kLLStride * j;
  r[0] = alpha * lam[j];
  for (int c = 1; c < kLLStride; ++c) r[c] = 0.0;
}

// One wavefront per mode j of the constant-H step: z_j = Ve[:, j] . y - eta_j
// (eta = Ve^T H s is carried in data space: H U0 = H P Ve and
// Ve^T H P Ve = Lambda, so the update s += U0 zp moves eta by Lambda zp),
// then the per-mode gain and D update, and the mode's log-likelihood terms.
__global__ void __launch_bounds__(256) k_modes_step_eta(const double *__restrict__ Ve, int n_m,
                                                        int nmode, const double *__restrict__ y,
                                                        const double *__restrict__ lam,
                                                        double *__restrict__ delta,
                                                        double *__restrict__ eta, double alpha,
                                                        double *__restrict__ zp,
                                                        double *__restrict__ llq, int *err) {
  int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nmode) return;
  int l = threadIdx.x & 63;
  // the mode's scalars are loaded before the dot product, so that their
  // latency overlaps it
  double *qj = llq + (int64_t)kLLStride * j;
  const double ej = eta[j], lj = lam[j], dj = delta[j];
  double q[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) q[c] = qj[c];
  const double *v = Ve + (int64_t)n_m * j;
  double z = 0;
  for (int m = l; m < n_m; m += 64) z = fma(v[m], y[m], z);
  z = wave_sum(z);
  if (l == 0) {
    z -= ej;
    double a = alpha - dj * lj;          // alpha_{k+1} - D_k
    double den = 1.0 + a * lj;           // (alpha - D) lambda + 1: S_k in the eigenbasis
    double g = a / den;
    double zpj = g * z;
    const double dn = dj + a * g;        // D_{k+1} / lambda
    zp[j] = zpj;
    delta[j] = dn;
    eta[j] = ej + lj * zpj;
    loglik_mode_step(q, a * lj, lj, z);
#pragma unroll
    for (int c = 0; c < 9; ++c) qj[c] = q[c];
    if (!isfinite(zpj) || !isfinite(dn)) atomicExch(err, (int)FKF_E_NONFINITE);
  }
}

// eta = Ve^T h (one wavefront per mode)
__global__ void __launch_bounds__(256) k_vet(const double *__restrict__ Ve, int n_m, int nmode,
                                             const double *__restrict__ h,
                                             double *__restrict__ eta) {
  int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nmode) return;
  int l = threadIdx.x & 63;
  const double *v = Ve + (int64_t)n_m * j;
  double z = 0;
  for (int m = l; m < n_m; m += 64) z = fma(v[m], h[m], z);
  z = wave_sum(z);
  if (l == 0) eta[j] = z;
}

// One wavefront per mode j: realization coefficients
// zz_j = (Ve[:, j] . h) * Sigma_-_j / lambda_j with Sigma_- = 1 - (1 - D/alpha)^1/2,
// written as (delta/alpha) / (1 + (1 - delta lambda / alpha)^1/2).
__global__ void __launch_bounds__(256) k_modes_realize(const double *__restrict__ Ve, int n_m,
                                                       int nmode, const double *__restrict__ h,
                                                       const double *__restrict__ lam,
                                                       const double *__restrict__ delta,
                                                       double alpha, double *__restrict__ zz) {
  int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nmode) return;
  int l = threadIdx.x & 63;
  const double *v = Ve + (int64_t)n_m * j;
  double z = 0;
  for (int m = l; m < n_m; m += 64) z = fma(v[m], h[m], z);
  z = wave_sum(z);
  if (l == 0) {
    double dl = delta[j] / alpha;
    double r = fmax(0.0, 1.0 - dl * lam[j]);
    zz[j] = z * dl / (1.0 + sqrt(r));
  }
}

// Row-panel GEMV with its epilogue, one launch and no partial sums:
// out_i = epilogue(sum_j f(U[i, j]) z[j]) with f(u) = u, or u^2 (SQUARE),
// for a column-major n x ncols basis (ld a multiple of 64, rows n..ld-1
// zero).  A workgroup of eight wavefronts owns one panel of kPanelRows rows
// (FP64: 128 rows, 2 per lane; FP32: 256 rows, 4 per lane, 16-byte loads);
// wavefront w streams the columns [w c, (w + 1) c) of the panel, eight
// loads in flight per lane (sixteen measured slower), and the eight partial sums of a row are added in
// wavefront order through LDS (fixed order: deterministic).  Epilogues:
//   kEpiAdd:     s_i += sum                        (state update)
//   kEpiVar:     out_i = base - sum                (variance)
//   kEpiRealize: out_i = s_i + salpha (g_i - sum)  (realization)
constexpr int kEpiAdd = 0, kEpiVar = 1, kEpiRealize = 2;
template <typename T> struct PanelRows;
template <> struct PanelRows<double> { static constexpr int v = 128; };
template <> struct PanelRows<float> { static constexpr int v = 256; };

template <typename T, int EPI, bool SQUARE>
__global__ void __launch_bounds__(512) k_gemv_panel(const T *__restrict__ U, int64_t n,
                                                    int64_t ldu, int ncols,
                                                    const double *__restrict__ z,
                                                    double *__restrict__ out,
                                                    const double *__restrict__ s,
                                                    const double *__restrict__ g, double base,
                                                    double salpha, const int *__restrict__ err,
                                                    int *__restrict__ err_mirror) {
  constexpr int R = 16 / sizeof(T);            // rows per lane (one 16-byte load)
  constexpr int PR = PanelRows<T>::v;          // rows per panel = 64 lanes x R
  typedef T vec __attribute__((ext_vector_type(R)));
  __shared__ double red[8][PR];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
  const int64_t r0 = (int64_t)blockIdx.x * PR;
  const int64_t i0 = r0 + (int64_t)R * l;
  if (EPI == kEpiAdd && err_mirror != nullptr && blockIdx.x == 0 && threadIdx.x == 0)
    *err_mirror = *err;   // latched device error, mirrored into pinned host memory
  const int cpw = (ncols + 7) / 8;
  const int j0 = w * cpw, j1 = min(ncols, j0 + cpw);
  double a[R];
#pragma unroll
  for (int h = 0; h < R; ++h) a[h] = 0.0;
  if (i0 < ldu && j0 < j1) {
    const vec *src = reinterpret_cast<const vec *>(U + i0 + ldu * (int64_t)j0);
    const int64_t ldv = ldu / R;
    auto acc = [&](vec u, double zj) {
#pragma unroll
      for (int h = 0; h < R; ++h) {
        const double x = (double)u[h];
        a[h] = SQUARE ? fma(x * x, zj, a[h]) : fma(x, zj, a[h]);
      }
    };
    int j = j0;
    for (; j + 8 <= j1; j += 8) {
      vec u[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) u[q] = __builtin_nontemporal_load(src + ldv * (j - j0 + q));
#pragma unroll
      for (int q = 0; q < 8; ++q) acc(u[q], z[j + q]);
    }
    for (; j < j1; ++j) acc(__builtin_nontemporal_load(src + ldv * (j - j0)), z[j]);
  }
#pragma unroll
  for (int h = 0; h < R; ++h) red[w][R * l + h] = a[h];
  __syncthreads();
  for (int t = threadIdx.x; t < PR; t += 512) {
    const int64_t i = r0 + t;
    if (i >= n) continue;
    double sum = red[0][t];
#pragma unroll
    for (int q = 1; q < 8; ++q) sum += red[q][t];
    if (EPI == kEpiAdd) out[i] += sum;
    else if (EPI == kEpiVar) out[i] = base - sum;
    else out[i] = s[i] + salpha * (g[i] - sum);
  }
}

__global__ void k_to_f32(const double *__restrict__ src, float *__restrict__ dst, int64_t len) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) dst[i] = (float)src[i];
}

// out[i] = s[i] + a g[i]
__global__ void k_axpy_out(const double *__restrict__ s, const double *__restrict__ g, double a,
                           double *__restrict__ out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = s[i] + a * g[i];
}

// h = H x (a sparse product used by the realization; no data vector)
__global__ void __launch_bounds__(256) k_spmv_f(const int64_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col,
                                                const double *__restrict__ val, int n_m,
                                                const double *__restrict__ x,
                                                double *__restrict__ h) {
  int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= n_m) return;
  int l = threadIdx.x & 63;
  double acc = 0;
  for (int64_t e = rowptr[m] + l; e < rowptr[m + 1]; e += 64) acc = fma(val[e], x[col[e]], acc);
  acc = wave_sum(acc);
  if (l == 0) h[m] = acc;
}

// Linearisation of the Box-Cox measurement model h(x) = H g(x) about the
// estimate x (extended filter, Algorithm 4; transform of eq. nonlinear):
// g(x) = t^a, g'(x) = t^(a-1), t = (x + a)/a, with t < 0 taken as 0 (g = 0,
// g' its one-sided limit: 1 for a = 1, else 0).  One wavefront per row m
// writes the row of H_k = H diag(g'(x)) (the sparsity of H) and
// ytil_m = y_m - sum_e H_e (g - g' x)_col(e), the data for which the linear
// update with H_k has innovation ytil - H_k x = y - h(x).  A non-finite
// estimate propagates into ytil and latches FKF_E_NONFINITE.
__global__ void __launch_bounds__(256) k_boxcox_linearize(const int64_t *__restrict__ rowptr,
                                                          const int32_t *__restrict__ col,
                                                          const double *__restrict__ val, int n_m,
                                                          const double *__restrict__ x, double a,
                                                          const double *__restrict__ y,
                                                          double *__restrict__ val_k,
                                                          double *__restrict__ ytil, int *err) {
  int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= n_m) return;
  int l = threadIdx.x & 63;
  const double edge = a == 1.0 ? 1.0 : 0.0;
  double acc = 0;
  for (int64_t e = rowptr[m] + l; e < rowptr[m + 1]; e += 64) {
    const double xi = x[col[e]];
    double t = (xi + a) / a;
    if (t < 0.0) t = 0.0;                      // NaN passes through
    const double gp = t > 0.0 ? pow(t, a - 1.0) : edge;
    const double g = t * gp;
    val_k[e] = val[e] * gp;
    acc = fma(val[e], g - gp * xi, acc);
  }
  acc = wave_sum(acc);
  if (l == 0) {
    double v = y[m] - acc;
    if (!isfinite(v)) atomicExch(err, (int)FKF_E_NONFINITE);
    ytil[m] = v;
  }
}

__global__ void k_set_flag(int *p, int v) { *p = v; }

__global__ void k_clamp_nonneg(double *__restrict__ x, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(x[i] > 0.0)) x[i] = 0.0;
}

__global__ void k_copy_strided(const double *__restrict__ src, double *__restrict__ dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Gaussian sketch of the randomized eigensolver (Appendix B), drawn on the
// device from a counter-based generator: Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, SC 2011; multipliers 0xD2511F53, 0xCD9E8D57, key increments
// 0x9E3779B9, 0xBB67AE85) of the counter (q mod 2^32, q div 2^32, 0, 0) under
// the key (seed mod 2^32, seed div 2^32), then the Box-Muller pair of the two
// 53-bit uniforms u1 = ((x0 >> 6) 2^27 + (x1 >> 5) + 1/2) 2^-53, u2 likewise:
// numbers 2q and 2q + 1 are sqrt(-2 ln u1) (cos, sin)(2 pi u2).  One thread
// per pair q.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    if (i > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)p1;
    c[2] = n2;
    c[3] = (uint32_t)p0;
  }
}

__global__ void k_sketch_normals(uint64_t seed, int64_t count, double *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * q >= count) return;
  uint32_t c[4] = {(uint32_t)q, (uint32_t)((uint64_t)q >> 32), 0u, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double sc = 1.0 / 9007199254740992.0;   // 2^-53
  const double u1 = ((double)(c[0] >> 6) * 134217728.0 + (double)(c[1] >> 5) + 0.5) * sc;
  const double u2 = ((double)(c[2] >> 6) * 134217728.0 + (double)(c[3] >> 5) + 0.5) * sc;
  const double rho = sqrt(-2.0 * log(u1));
  const double t = 2.0 * M_PI * u2;
  out[2 * q] = rho * cos(t);
  if (2 * q + 1 < count) out[2 * q + 1] = rho * sin(t);
}

// --------------------------------------------------------------- helpers ---
static unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// out = epilogue(f(M) z) for a column-major n x ncols matrix M (ld a multiple
// of 64) in FP64 or FP32 (k_gemv_panel).
struct GemvEpi {
  int kind = kEpiAdd;
  const double *s = nullptr, *g = nullptr;
  double base = 0.0, salpha = 0.0;
  const int *err = nullptr;
  int *err_mirror = nullptr;
};

template <typename T>
static void gemv_panel_t(const T *M, int64_t ld, int ncols, int64_t n, const double *z,
                         bool square, double *out, const GemvEpi &e, hipStream_t st) {
  const unsigned grid = (unsigned)((ld + PanelRows<T>::v - 1) / PanelRows<T>::v);
  if (grid == 0) return;
#define FKF_GEMV_LAUNCH(EPI, SQ)                                                            \
  hipLaunchKernelGGL((k_gemv_panel<T, EPI, SQ>), dim3(grid), dim3(512), 0, st, M, n, ld, ncols, \
                     z, out, e.s, e.g, e.base, e.salpha, e.err, e.err_mirror)
  if (e.kind == kEpiAdd) {
    if (square) FKF_GEMV_LAUNCH(kEpiAdd, true);
    else FKF_GEMV_LAUNCH(kEpiAdd, false);
  } else if (e.kind == kEpiVar) {
    if (square) FKF_GEMV_LAUNCH(kEpiVar, true);
    else FKF_GEMV_LAUNCH(kEpiVar, false);
  } else {
    if (square) FKF_GEMV_LAUNCH(kEpiRealize, true);
    else FKF_GEMV_LAUNCH(kEpiRealize, false);
  }
#undef FKF_GEMV_LAUNCH
}

static void gemv_panel_m(const double *M, int64_t ld, int ncols, int64_t n, const double *z,
                         bool square, double *out, const GemvEpi &e, hipStream_t st) {
  FKF_TRACE(square ? "filter_gemv_sq" : "filter_gemv", st);
  gemv_panel_t<double>(M, ld, ncols, n, z, square, out, e, st);
}

// The same over the filter's constant-H basis U0 (its FP32 copy in the mixed
// mode).
static void gemv_panel(const fkf_filter *f, const double *z, bool square, double *out,
                       const GemvEpi &e, hipStream_t st) {
  if (f->mixed) {
    FKF_TRACE(square ? "filter_gemv_sq32" : "filter_gemv32", st);
    gemv_panel_t<float>(f->U0f.p, f->ldu, f->nmode, f->n, z, square, out, e, st);
    return;
  }
  gemv_panel_m(f->U0.p, f->ldu, f->nmode, f->n, z, square, out, e, st);
}

// Stopping tolerance of the projected generalized eigenproblem (relative
// off-diagonal norm): 1e-12 in FP64; 1e-10 for a mixed-precision filter,
// whose FP32 storage already perturbs the results by ~1e-7 relative.
static double gep_tol(const fkf_filter *f) { return f->mixed ? 1e-10 : 1e-12; }

// P = Gamma H^T (n x n_m, leading dimension ldp): the several-column product
// taking its columns as the sparse rows of H where that form applies, else
// the product with the dense H^T (in Ht: formed here unless ht_ready).
static void cross_cov(fkf_cov *cov, const fkf_obs *o, DevBuf<double> &Ht, double *P,
                      int64_t ldp, hipStream_t st, bool ht_ready = false) {
  const int64_t n = o->n;
  if (cov_apply_sparse_rows(cov, o->n_m, o->rowptr.p, o->col.p, o->val.p, o->nnz, o->max_row,
                            o->order.p, P, ldp, st))
    return;
  if (!ht_ready) {
    Ht.reserve((size_t)n * o->n_m);
    dense_ht(o->rowptr.p, o->col.p, o->val.p, o->n_m, n, Ht.p, st);
  }
  fkf_status rc = fkf_cov_apply(cov, Ht.p, n, o->n_m, P, ldp, (void *)st);
  if (rc != FKF_OK) throw Error{rc, std::string("covariance product failed: ") + fkf_last_error()};
}

// Rayleigh-Ritz for the generalized eigenproblem H^T R^-1 H x = lambda Gamma^-1 x
// on range(Gamma H^T): P = Gamma H^T (H-matrix product), G = H P, and the
// eigenpairs (lam descending, We) of A = R^-1/2 sym(G) R^-1/2.  Ht holds the
// dense H^T (the dual of P's range).  Negative rounding-level eigenvalues are
// set to zero.
static void compute_gep(fkf_filter *f, const fkf_obs *o, DevBuf<double> &Ht, DevBuf<double> &P,
                        DevBuf<double> &G, DevBuf<double> &A, DevBuf<double> &lam,
                        DevBuf<double> &We, hipStream_t st) {
  const int64_t n = f->n;
  const int nm = o->n_m;
  P.reserve((size_t)n * nm);
  G.reserve((size_t)nm * nm);
  A.reserve((size_t)nm * nm);
  lam.reserve(nm);
  We.reserve((size_t)nm * nm);
  Ht.reserve((size_t)n * nm);   // the dense H^T, also used after the eigensolve
  dense_ht(o->rowptr.p, o->col.p, o->val.p, nm, n, Ht.p, st);
  {
    FKF_TRACE("gep_cross_cov", st);
    cross_cov(f->cov, o, Ht, P.p, n, st, true);
  }
  innovation_gram(o->rowptr.p, o->col.p, o->val.p, nm, n, P.p, o->noise.p, G.p, A.p, st);
  {
    FKF_TRACE("gep_eig", st);
    sym_eig(A.p, nm, nm, lam.p, We.p, nm, st, f->eig, gep_tol(f), f->err.p);
  }
  hipLaunchKernelGGL(k_clamp_nonneg, dim3(blocks(nm)), dim3(256), 0, st, lam.p, nm);
}

// Constant-H basis U0 = P R^-1/2 W_e (the generalized eigenvectors times
// Lambda^1/2), Ve = R^-1/2 W_e, lambda; delta = D / lambda starts at zero.
// Streams (default priority) over which the work of independent filters is
// spread, and the fork/join between them and the caller's stream: lane c of
// a fork runs on pool stream c after everything queued on the caller's
// stream so far; the join makes the caller's stream wait for every lane.
constexpr int kLanes = 4;
struct LanePool {
  hipStream_t s[kLanes] = {};
  hipEvent_t fork = nullptr, join[kLanes] = {};
};

static LanePool &lane_pool() {
  static std::mutex mu;
  static std::map<int, LanePool> pools;   // per device
  int dev = 0;
  FKF_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  LanePool &p = pools[dev];
  if (!p.fork) {
    for (int c = 0; c < kLanes; ++c) {
      FKF_CHECK_HIP(hipStreamCreateWithFlags(&p.s[c], hipStreamNonBlocking));
      FKF_CHECK_HIP(hipEventCreateWithFlags(&p.join[c], hipEventDisableTiming));
    }
    FKF_CHECK_HIP(hipEventCreateWithFlags(&p.fork, hipEventDisableTiming));
  }
  return p;
}

static void lanes_fork(LanePool &p, hipStream_t st) {
  FKF_CHECK_HIP(hipEventRecord(p.fork, st));
  for (int c = 0; c < kLanes; ++c) FKF_CHECK_HIP(hipStreamWaitEvent(p.s[c], p.fork, 0));
}

static void lanes_join(LanePool &p, hipStream_t st) {
  for (int c = 0; c < kLanes; ++c) {
    FKF_CHECK_HIP(hipEventRecord(p.join[c], p.s[c]));
    FKF_CHECK_HIP(hipStreamWaitEvent(st, p.join[c], 0));
  }
}

// Lane of each filter: filters that use a common operator (their covariance
// or their length-derivative operator, whose product workspaces are not
// reentrant) share a lane.  Filters are joined into groups through every
// operator they use (union-find), and each group takes one lane.
static std::vector<int> lanes_of(fkf_filter *const *fs, int count) {
  std::vector<int> up(count);
  for (int i = 0; i < count; ++i) up[i] = i;
  auto root = [&](int i) {
    while (up[i] != i) i = up[i] = up[up[i]];
    return i;
  };
  std::map<const fkf_cov *, int> owner;   // operator -> a filter that uses it
  for (int i = 0; i < count; ++i)
    for (const fkf_cov *c : {(const fkf_cov *)fs[i]->cov, (const fkf_cov *)fs[i]->dcov}) {
      if (!c) continue;
      auto it = owner.find(c);
      if (it == owner.end()) owner.emplace(c, i);
      else up[root(i)] = root(it->second);
    }
  std::map<int, int> group_lane;
  std::vector<int> lane(count);
  for (int i = 0; i < count; ++i) {
    auto it = group_lane.find(root(i));
    if (it == group_lane.end())
      it = group_lane.emplace(root(i), (int)group_lane.size() % kLanes).first;
    lane[i] = it->second;
  }
  return lane;
}

static std::vector<double> to_host(const double *p, size_t n, hipStream_t st) {
  std::vector<double> h(n);
  if (n) {
    FKF_CHECK_HIP(hipMemcpyAsync(h.data(), p, n * sizeof(double), hipMemcpyDeviceToHost, st));
    FKF_CHECK_HIP(hipStreamSynchronize(st));
  }
  return h;
}

static void upload_vec(DevBuf<double> &d, const std::vector<double> &h, hipStream_t st) {
  d.reserve(std::max<size_t>(h.size(), 1));
  d.upload(h.data(), h.size(), st);
}

// Number of leading (descending) values strictly above thr.
static int count_above(const std::vector<double> &v, double thr) {
  int r = 0;
  while (r < (int)v.size() && v[r] > thr) ++r;
  return r;
}

// The part of a constant-H basis build shared by the exact and the
// randomized eigensolver, once lam (nmode modes, descending), Ve (n_m x nmode)
// and U0 (n x nmode, ld ldu) are in place: the FP32 copy of the basis, the
// carriers delta = 0, the per-mode log-likelihood state, a copy of the
// operator and eta = Ve^T H s for the current estimate.
static void basis_tail(fkf_filter *f, const fkf_obs *o, int nmode, hipStream_t si) {
  const int nm = o->n_m;
  f->n_m = nm;
  f->nmode = nmode;
  if (f->mixed) {
    f->U0f.reserve((size_t)f->ldu * nmode);
    const int64_t len = f->ldu * (int64_t)nmode;
    if (len > 0)
      hipLaunchKernelGGL(k_to_f32, dim3(blocks(len)), dim3(256), 0, si, f->U0.p, f->U0f.p, len);
  }
  f->llq.reserve((size_t)kLLStride * nmode);
  hipLaunchKernelGGL(k_loglik_init, dim3(blocks(nmode)), dim3(256), 0, si, f->llq.p, f->lam.p,
                     nmode, f->alpha);
  f->delta.reserve(nmode);
  fill(f->delta.p, nmode, 0.0, si);
  f->nu.reserve(std::max(nm, nmode));
  f->zp.reserve(nmode);
  f->tmp.reserve(nmode);
  f->b_rowptr.copy_into(o->rowptr.p, (size_t)nm + 1, si);
  f->b_col.copy_into(o->col.p, (size_t)o->nnz, si);
  f->b_val.copy_into(o->val.p, (size_t)o->nnz, si);
  f->eta.reserve(nmode);
  spmv(o->rowptr.p, o->col.p, o->val.p, nm, f->s.p, f->nu.p, si);
  hipLaunchKernelGGL(k_vet, dim3(blocks(nmode, 4)), dim3(256), 0, si, f->Ve.p, nm, nmode, f->nu.p,
                     f->eta.p);
  f->mode = 1;
  f->basis_gen = o->gen;
}

// Constant-H bases of count filters (filter i with operator obs[i]): the
// cross covariances, innovation Grams and, after one batched eigensolve of
// the projected problems, the bases and carriers.  With several filters the
// per-filter work runs on kLanes streams (joined before the eigensolve and
// at the end).
static void build_bases(fkf_filter *const *fs, const fkf_obs *const *os, int count,
                        hipStream_t st) {
  FKF_TRACE("gep_total", st);
  std::vector<EigProblem> probs(count);
  int nbatch = 0;
  double tol = 1.0;
  const bool multi = count > 1;
  LanePool *lp = multi ? &lane_pool() : nullptr;
  const std::vector<int> lane = lanes_of(fs, count);
  auto sti = [&](int i) { return multi ? lp->s[lane[i]] : st; };
  if (multi) lanes_fork(*lp, st);
  for (int i = 0; i < count; ++i) {
    fkf_filter *f = fs[i];
    const fkf_obs *o = os[i];
    const int64_t n = f->n;
    const int nm = o->n_m;
    hipStream_t si = sti(i);
    fs[i]->bw.P.reserve((size_t)n * nm);
    fs[i]->bw.G.reserve((size_t)nm * nm);
    fs[i]->bw.A.reserve((size_t)nm * nm);
    f->lam.reserve(nm);
    f->Ve.reserve((size_t)nm * nm);
    {
      FKF_TRACE("gep_cross_cov", si);
      cross_cov(f->cov, o, fs[i]->bw.Ht, fs[i]->bw.P.p, n, si);
    }
    innovation_gram(o->rowptr.p, o->col.p, o->val.p, nm, n, fs[i]->bw.P.p, o->noise.p, fs[i]->bw.G.p,
                    fs[i]->bw.A.p, si);
    if (multi && sym_eig_dc_supported(nm)) {
      // the divide-and-conquer solver per filter, on the filter's lane (up
      // to one reduction per lane at a time: their workgroups fit the chip
      // together, so the reductions' waits always end)
      FKF_TRACE("gep_eig", si);
      sym_eig(fs[i]->bw.A.p, nm, nm, f->lam.p, f->Ve.p, nm, si, f->eig, gep_tol(f), f->err.p);
    } else {
      probs[nbatch] = EigProblem{fs[i]->bw.A.p, nm, nm, 0, f->lam.p, f->Ve.p, nm};
      tol = std::min(tol, gep_tol(f));
      ++nbatch;
    }
  }
  if (multi) lanes_join(*lp, st);
  if (nbatch > 0) {
    // other orders (and a single filter) as one batch
    FKF_TRACE("gep_eig", st);
    sym_eig_batched(probs.data(), nbatch, st, fs[0]->eig, tol, fs[0]->err.p);
  }
  if (multi) lanes_fork(*lp, st);
  for (int i = 0; i < count; ++i) {
    fkf_filter *f = fs[i];
    const fkf_obs *o = os[i];
    const int64_t n = f->n;
    const int nm = o->n_m;
    hipStream_t si = sti(i);
    hipLaunchKernelGGL(k_clamp_nonneg, dim3(blocks(nm)), dim3(256), 0, si, f->lam.p, nm);
    scale_rows(nm, nm, o->inv_sqrt_noise.p, f->Ve.p, nm, si);
    f->ldu = (n + 63) / 64 * 64;
    f->U0.reserve((size_t)f->ldu * nm);
    fill(f->U0.p, f->ldu * nm, 0.0, si);
    {
      FKF_TRACE("gep_basis_gemm", si);
      gemm_nn(n, nm, nm, fs[i]->bw.P.p, n, f->Ve.p, nm, f->U0.p, f->ldu, si);
    }
    if (f->dcov) {
      // Ad = Ve^T H (dGamma/d ell) H^T Ve: the derivative operator applied to
      // the sparse rows of H as for the cross covariance (P, free once the
      // basis GEMM above has read it), G' = H (dGamma/d ell) H^T from its
      // upper triangle, then Ad = Ve^T G' Ve; Cd starts at alpha Ad
      FKF_TRACE("loglik_length_setup", si);
      cross_cov(f->dcov, o, fs[i]->bw.Ht, fs[i]->bw.P.p, n, si);
      innovation_gram(o->rowptr.p, o->col.p, o->val.p, nm, n, fs[i]->bw.P.p, o->noise.p,
                      fs[i]->bw.G.p, fs[i]->bw.A.p, si);
      gemm(false, false, nm, nm, nm, 1.0, fs[i]->bw.G.p, nm, f->Ve.p, nm, 0.0, fs[i]->bw.A.p, nm,
           si, &f->gwork);
      f->ll_Ad.reserve((size_t)nm * nm);
      f->ll_Cd.reserve((size_t)nm * nm);
      gemm(true, false, nm, nm, nm, 1.0, f->Ve.p, nm, fs[i]->bw.A.p, nm, 0.0, f->ll_Ad.p, nm, si,
           &f->gwork);
      symmetrize(f->ll_Ad.p, nm, si);
      copy2d(nm, nm, f->ll_Ad.p, nm, f->ll_Cd.p, nm, si);
      scale2d(nm, nm, f->alpha, f->ll_Cd.p, nm, si);
    }
    basis_tail(f, o, nm, si);
  }
  if (multi) lanes_join(*lp, st);
}

// Constant-H basis by the randomized algorithm of Appendix B (one filter):
// Omega (n x r, r = k + p) from the sketch stream; M = R^-1 H Omega and
// Ybar = H^T M (A Omega with A = H^T R^-1 H); Z = Gamma Ybar (an r-column
// H-matrix product); a Gamma-orthonormal basis of range(Ybar) from two
// passes of Gram eigen-decompositions (Gram = Ybar^T Z, directions with
// eigenvalue <= 1e-12 of the largest dropped, then the same once more on the
// result), i.e. Qhat = Ybar C with Qhat^T Gamma Qhat = I and Q = Z C;
// T = (H Q)^T R^-1 (H Q) = S Lambda S^T; the k largest modes with
// lambda > 1e-13 lambda_max give U = Q S_k, stored as U0 = U Lambda^1/2 and
// Ve = R^-1 H U Lambda^-1/2 (so that the constant-H step projects the data
// with Ve exactly as in the exact form).
static void build_basis_randomized(fkf_filter *f, const fkf_obs *o, hipStream_t st) {
  FKF_TRACE("gep_total", st);
  const int64_t n = f->n;
  const int nm = o->n_m;
  const int k = f->params.gep_rank > 0 ? std::min(f->params.gep_rank, nm) : nm;
  const int r = (int)std::min<int64_t>((int64_t)k + f->params.oversample, n);
  BasisWork &w = f->bw;
  w.X.reserve((size_t)n * r);   // Omega, then Ybar C1
  w.P.reserve((size_t)n * r);   // Ybar
  w.Ht.reserve((size_t)n * nm);
  DevBuf<double> &Z = f->gP, &HZ = f->gG, &sm = f->gA;   // reused general-step workspaces
  Z.reserve((size_t)n * r);
  HZ.reserve((size_t)nm * r);
  // small r x r work: M (nm x r), G1, V1, C1, G2, V2, C, HQ (nm x r), T, S
  const size_t rr = (size_t)r * r;
  sm.reserve(8 * rr + 2 * (size_t)nm * r + 4 * (size_t)r);
  double *M = sm.p, *G1 = M + (size_t)nm * r, *V1 = G1 + rr, *C1 = V1 + rr, *G2 = C1 + rr,
         *V2 = G2 + rr, *C = V2 + rr, *HQ = C + rr, *T = HQ + (size_t)nm * r, *S = T + rr,
         *ev = S + rr;
  {
    FKF_TRACE("gep_sketch", st);
    const int64_t cnt = n * (int64_t)r;
    hipLaunchKernelGGL(k_sketch_normals, dim3(blocks((cnt + 1) / 2)), dim3(256), 0, st,
                       f->params.seed, cnt, w.X.p);
    sp_dense(o->rowptr.p, o->col.p, o->val.p, nm, w.X.p, n, r, M, st);
    scale_rows(nm, r, o->inv_sqrt_noise.p, M, nm, st);
    scale_rows(nm, r, o->inv_sqrt_noise.p, M, nm, st);
    dense_ht(o->rowptr.p, o->col.p, o->val.p, nm, n, w.Ht.p, st);
    gemm_nn(n, r, nm, w.Ht.p, n, M, nm, w.P.p, n, st);
  }
  {
    FKF_TRACE("gep_cross_cov", st);
    fkf_status rc = fkf_cov_apply(f->cov, w.P.p, n, r, Z.p, n, (void *)st);
    if (rc != FKF_OK) throw Error{rc, std::string("covariance product failed: ") + fkf_last_error()};
  }
  FKF_TRACE("gep_eig", st);
  // first pass: Gram = Ybar^T Gamma Ybar = Q1 Theta Q1^T, C1 = Q1 Theta^-1/2
  gemm(true, false, r, r, n, 1.0, w.P.p, n, Z.p, n, 0.0, G1, r, st, &f->gwork);
  symmetrize(G1, r, st);
  sym_eig(G1, r, r, ev, V1, r, st, f->eig, 1e-12, f->err.p);
  std::vector<double> th = to_host(ev, r, st);
  const int r1 = count_above(th, 1e-12 * (th.empty() ? 0.0 : th[0]));
  if (r1 == 0) throw Error{FKF_E_RANK, "fkf_filter_step: the sketch of H^T R^-1 H is zero"};
  std::vector<double> ith(r1);
  for (int j = 0; j < r1; ++j) ith[j] = 1.0 / std::sqrt(th[j]);
  DevBuf<double> s_i;
  upload_vec(s_i, ith, st);
  copy2d(r, r1, V1, r, C1, r, st);
  scale_cols(r, r1, s_i.p, C1, r, st);
  // second pass on Qhat1 = Ybar C1, Q1 = Z C1: Gram2 = C1^T (Ybar^T Z) C1 recomputed from the
  // vectors (Qhat1^T Q1), so that the rounding of the first pass is removed
  gemm_nn(n, r1, r, w.P.p, n, C1, r, w.X.p, n, st);                // Qhat1 (in X)
  gemm_nn(n, r1, r, Z.p, n, C1, r, w.Ht.p, n, st);                 // Q1 (in Ht, n x r1 <= n x nm?)
  gemm(true, false, r1, r1, n, 1.0, w.X.p, n, w.Ht.p, n, 0.0, G2, r1, st, &f->gwork);
  symmetrize(G2, r1, st);
  sym_eig(G2, r1, r1, ev, V2, r1, st, f->eig, 1e-12, f->err.p);
  std::vector<double> th2 = to_host(ev, r1, st);
  const int r2 = count_above(th2, 1e-12 * (th2.empty() ? 0.0 : th2[0]));
  std::vector<double> ith2(r2);
  for (int j = 0; j < r2; ++j) ith2[j] = 1.0 / std::sqrt(th2[j]);
  upload_vec(s_i, ith2, st);
  scale_cols(r1, r2, s_i.p, V2, r1, st);
  gemm_nn(r, r2, r1, C1, r, V2, r1, C, r, st);                    // C = C1 V2 Theta2^-1/2
  // T = (H Q)^T R^-1 (H Q) with H Q = (H Z) C, whitened: B = R^-1/2 H Q (in HQ)
  sp_dense(o->rowptr.p, o->col.p, o->val.p, nm, Z.p, n, r, HZ.p, st);
  gemm_nn(nm, r2, r, HZ.p, nm, C, r, HQ, nm, st);
  scale_rows(nm, r2, o->inv_sqrt_noise.p, HQ, nm, st);
  gemm(true, false, r2, r2, nm, 1.0, HQ, nm, HQ, nm, 0.0, T, r2, st, &f->gwork);
  symmetrize(T, r2, st);
  sym_eig(T, r2, r2, ev, S, r2, st, f->eig, gep_tol(f), f->err.p);
  std::vector<double> lam = to_host(ev, r2, st);
  const int kk = std::min(k, count_above(lam, 1e-13 * (lam.empty() ? 0.0 : lam[0])));
  if (kk == 0) throw Error{FKF_E_RANK, "fkf_filter_step: the operator carries no information"};
  lam.resize(kk);
  std::vector<double> sl(kk), isl(kk);
  for (int j = 0; j < kk; ++j) {
    sl[j] = std::sqrt(lam[j]);
    isl[j] = 1.0 / sl[j];
  }
  // U0 = Z (C S_k Lambda^1/2), Ve = R^-1/2 (B S_k) Lambda^-1/2
  f->lam.reserve(kk);
  FKF_CHECK_HIP(hipMemcpyAsync(f->lam.p, lam.data(), kk * sizeof(double), hipMemcpyHostToDevice, st));
  DevBuf<double> s_l, CS((size_t)r * kk);
  upload_vec(s_l, sl, st);
  gemm_nn(r, kk, r2, C, r, S, r2, CS.p, r, st);
  scale_cols(r, kk, s_l.p, CS.p, r, st);
  f->ldu = (n + 63) / 64 * 64;
  f->U0.reserve((size_t)f->ldu * kk);
  fill(f->U0.p, f->ldu * kk, 0.0, st);
  {
    FKF_TRACE("gep_basis_gemm", st);
    gemm_nn(n, kk, r, Z.p, n, CS.p, r, f->U0.p, f->ldu, st);
  }
  f->Ve.reserve((size_t)nm * kk);
  gemm_nn(nm, kk, r2, HQ, nm, S, r2, f->Ve.p, nm, st);
  upload_vec(s_l, isl, st);
  scale_cols(nm, kk, s_l.p, f->Ve.p, nm, st);
  scale_rows(nm, kk, o->inv_sqrt_noise.p, f->Ve.p, nm, st);
  basis_tail(f, o, kk, st);
  FKF_CHECK_HIP(hipStreamSynchronize(st));   // the small host-uploaded vectors are released
}

static void build_basis(fkf_filter *f, const fkf_obs *o, hipStream_t st) {
  if (f->params.gep_mode == FKF_GEP_RANDOMIZED) build_basis_randomized(f, o, st);
  else build_bases(&f, &o, 1, st);
}

// Constant-H form -> general form: W = U0 Lambda^-1/2 (= U), Wd = H_b^T Ve
// Lambda^-1/2 (= Gamma^-1 U), D = delta lambda, keeping the modes with
// lambda > 1e-13 lambda_max (the others carry Gamma^-1-norm sqrt(lambda)).
static void to_general(fkf_filter *f, hipStream_t st) {
  const int64_t n = f->n;
  const int nm = f->n_m;
  std::vector<double> lam = to_host(f->lam.p, f->nmode, st), del = to_host(f->delta.p, f->nmode, st);
  const int r = count_above(lam, 1e-13 * (lam.empty() ? 0.0 : lam[0]));
  std::vector<double> isl(r), dg(r);
  for (int j = 0; j < r; ++j) {
    isl[j] = 1.0 / std::sqrt(lam[j]);
    dg[j] = del[j] * lam[j];
  }
  DevBuf<double> s_isl;
  upload_vec(s_isl, isl, st);
  f->W.alloc((size_t)f->ldu * std::max(r, 1));
  f->Wd.alloc((size_t)f->ldu * std::max(r, 1));
  copy2d(n, r, f->U0.p, f->ldu, f->W.p, f->ldu, st);
  scale_cols(n, r, s_isl.p, f->W.p, f->ldu, st);
  DevBuf<double> Hbt((size_t)n * nm);
  dense_ht(f->b_rowptr.p, f->b_col.p, f->b_val.p, nm, n, Hbt.p, st);
  gemm(false, false, n, r, nm, 1.0, Hbt.p, n, f->Ve.p, nm, 0.0, f->Wd.p, f->ldu, st, nullptr);
  scale_cols(n, r, s_isl.p, f->Wd.p, f->ldu, st);
  upload_vec(f->Dg, dg, st);
  f->rg = r;
  f->mode = 2;
  FKF_CHECK_HIP(hipStreamSynchronize(st));
}

__global__ void k_general_coefs(const double *__restrict__ D, int r, double alpha,
                                const double *__restrict__ HWt, int nm, double *__restrict__ T) {
  // T (r x nm) = diag(D) (H W)^T, HWt holds H W (nm x r)
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)r * nm) return;
  int j = (int)(e % r), m = (int)(e / r);
  T[j + (int64_t)r * m] = D[j] * HWt[m + (int64_t)nm * j];
}

// x[i] += d[i]
__global__ void k_add_vec(double *__restrict__ x, const double *__restrict__ d, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += d[i];
}

__global__ void k_add_diag(double *__restrict__ S, int m, const double *__restrict__ d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) S[i + (int64_t)m * i] += d[i];
}

// Realization coefficients of the general form: zz_j = z_j Sigma_-_j with
// Sigma_- = 1 - (1 - D/alpha)^1/2 = (D/alpha) / (1 + (1 - D/alpha)^1/2).
__global__ void k_sigma_minus(const double *__restrict__ D, const double *__restrict__ z, int r,
                              double alpha, double *__restrict__ zz) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  double x = D[j] / alpha;
  zz[j] = z[j] * x / (1.0 + sqrt(fmax(0.0, 1.0 - x)));
}

// One step of the general form (Section 2.4 with Algorithm 5).
static void step_general(fkf_filter *f, const fkf_obs *o, const double *y, hipStream_t st) {
  FKF_TRACE("general_step", st);
  const int64_t n = f->n, ldu = f->ldu;
  const int nm = o->n_m;
  const int r = f->rg;
  const double a1 = f->alpha + 1.0;
  DevBuf<double> &P = f->gP, &Ht = f->gHt, &G = f->gG, &A = f->gA, &We = f->gWe, &lam = f->glam;
  {
    FKF_TRACE("general_gep", st);
    compute_gep(f, o, Ht, P, G, A, lam, We, st);
  }
  // eigenpairs with lambda > 1e-13 lambda_max: Z = R^-1/2 We Lambda^-1/2, U = P Z, Ud = H^T Z
  std::vector<double> lh = to_host(lam.p, nm, st);
  const int rk = count_above(lh, 1e-13 * (lh.empty() ? 0.0 : lh[0]));
  std::vector<double> isl(rk);
  for (int j = 0; j < rk; ++j) isl[j] = 1.0 / std::sqrt(lh[j]);
  DevBuf<double> s_isl, Z((size_t)nm * std::max(rk, 1));
  upload_vec(s_isl, isl, st);
  copy2d(nm, rk, We.p, nm, Z.p, nm, st);
  scale_rows(nm, rk, o->inv_sqrt_noise.p, Z.p, nm, st);
  scale_cols(nm, rk, s_isl.p, Z.p, nm, st);
  DevBuf<double> U((size_t)ldu * std::max(rk, 1)), Ud((size_t)ldu * std::max(rk, 1));
  gemm(false, false, n, rk, nm, 1.0, P.p, n, Z.p, nm, 0.0, U.p, ldu, st, nullptr);
  gemm(false, false, n, rk, nm, 1.0, Ht.p, n, Z.p, nm, 0.0, Ud.p, ldu, st, nullptr);
  // gain: F = a1 P - W diag(D) (H W)^T ; S = a1 G - (H W) diag(D) (H W)^T + R
  DevBuf<double> F((size_t)n * nm), S((size_t)nm * nm), HW((size_t)nm * std::max(r, 1)),
      T((size_t)std::max(r, 1) * nm), c(nm);
  copy2d(n, nm, P.p, n, F.p, n, st);
  copy2d(nm, nm, G.p, nm, S.p, nm, st);
  if (r > 0) {
    sp_dense(o->rowptr.p, o->col.p, o->val.p, nm, f->W.p, ldu, r, HW.p, st);
    hipLaunchKernelGGL(k_general_coefs, dim3(blocks((int64_t)r * nm)), dim3(256), 0, st, f->Dg.p,
                       r, a1, HW.p, nm, T.p);
    gemm(false, false, n, nm, r, -1.0, f->W.p, ldu, T.p, r, a1, F.p, n, st, nullptr);
    gemm(false, false, nm, nm, r, -1.0, HW.p, nm, T.p, r, a1, S.p, nm, st, nullptr);
  } else {
    scale2d(n, nm, a1, F.p, n, st);
    scale2d(nm, nm, a1, S.p, nm, st);
  }
  symmetrize(S.p, nm, st);
  hipLaunchKernelGGL(k_add_diag, dim3(blocks(nm)), dim3(256), 0, st, S.p, nm, o->noise.p);
  // state: c = S^-1 (y - H s), s += F c
  hipLaunchKernelGGL(k_innov, dim3(blocks(nm, 4)), dim3(256), 0, st, o->rowptr.p, o->col.p,
                     o->val.p, nm, f->s.p, y, c.p, f->err.p);
  f->chol_flag.reserve(1);
  if (!f->ll_gen.p) {
    f->ll_gen.alloc(1);
    fill(f->ll_gen.p, 1, 0.0, st);
  }
  f->gll.reserve(1);
  fill(f->gll.p, 1, 0.0, st);
  chol_solve(S.p, nm, c.p, f->chol_flag.p, f->err.p, st, f->gll.p);
  f->gdv.reserve((size_t)n);
  gemm(false, false, n, 1, nm, 1.0, F.p, n, c.p, nm, 0.0, f->gdv.p, n, st, nullptr);
  // covariance: Dbar = D / (a1 (a1 - D)); AddLowRank(W, Dbar, U, Lambda; Gamma^-1)
  std::vector<double> dh = to_host(f->Dg.p, r, st);
  std::vector<double> dbar(r);
  for (int j = 0; j < r; ++j) dbar[j] = dh[j] / (a1 * (a1 - dh[j]));
  DevBuf<double> C((size_t)std::max(r, 1) * std::max(rk, 1));
  DevBuf<double> Vt((size_t)ldu * std::max(rk, 1)), Vtd((size_t)ldu * std::max(rk, 1));
  copy2d(n, rk, U.p, ldu, Vt.p, ldu, st);
  copy2d(n, rk, Ud.p, ldu, Vtd.p, ldu, st);
  if (r > 0) {
    // C = W^T Gamma^-1 U = Wd^T U; Vt = U - W C (block Gram-Schmidt), dual likewise
    gemm(true, false, r, rk, n, 1.0, f->Wd.p, ldu, U.p, ldu, 0.0, C.p, r, st, &f->gwork);
    gemm(false, false, n, rk, r, -1.0, f->W.p, ldu, C.p, r, 1.0, Vt.p, ldu, st, nullptr);
    gemm(false, false, n, rk, r, -1.0, f->Wd.p, ldu, C.p, r, 1.0, Vtd.p, ldu, st, nullptr);
  }
  // Gamma^-1-orthonormal basis of Vt: Gram = Vtd^T Vt = Q Theta Q^T, keep theta > 1e-12
  DevBuf<double> Gm((size_t)std::max(rk, 1) * std::max(rk, 1)), th(std::max(rk, 1)),
      Q((size_t)std::max(rk, 1) * std::max(rk, 1));
  gemm(true, false, rk, rk, n, 1.0, Vtd.p, ldu, Vt.p, ldu, 0.0, Gm.p, rk, st, &f->gwork);
  symmetrize(Gm.p, rk, st);
  {
    FKF_TRACE("general_gram_eig", st);
    sym_eig(Gm.p, rk, rk, th.p, Q.p, rk, st, f->eig, 1e-12, f->err.p);
  }
  std::vector<double> thh = to_host(th.p, rk, st);
  const int rp = count_above(thh, 1e-12);
  std::vector<double> ith(rp);
  for (int j = 0; j < rp; ++j) ith[j] = 1.0 / std::sqrt(thh[j]);
  DevBuf<double> s_ith;
  upload_vec(s_ith, ith, st);
  scale_cols(rk, rp, s_ith.p, Q.p, rk, st);                 // Q Theta^-1/2
  const int rt = r + rp;
  DevBuf<double> Wc((size_t)ldu * std::max(rt, 1)), Wcd((size_t)ldu * std::max(rt, 1));
  copy2d(n, r, f->W.p, ldu, Wc.p, ldu, st);
  copy2d(n, r, f->Wd.p, ldu, Wcd.p, ldu, st);
  gemm(false, false, n, rp, rk, 1.0, Vt.p, ldu, Q.p, rk, 0.0, Wc.p + ldu * r, ldu, st, nullptr);
  gemm(false, false, n, rp, rk, 1.0, Vtd.p, ldu, Q.p, rk, 0.0, Wcd.p + ldu * r, ldu, st, nullptr);
  // B1 = [C; Vh^T Gamma^-1 U] (rt x rk), M = diag(Dbar, 0) + B1 Lambda B1^T
  DevBuf<double> B1((size_t)std::max(rt, 1) * std::max(rk, 1)), B1L((size_t)std::max(rt, 1) * std::max(rk, 1)),
      M((size_t)std::max(rt, 1) * std::max(rt, 1));
  copy2d(r, rk, C.p, r, B1.p, rt, st);
  gemm(true, false, rp, rk, n, 1.0, Wcd.p + ldu * r, ldu, U.p, ldu, 0.0, B1.p + r, rt, st,
       &f->gwork);
  std::vector<double> lamk(lh.begin(), lh.begin() + rk);
  DevBuf<double> s_lam;
  upload_vec(s_lam, lamk, st);
  copy2d(rt, rk, B1.p, rt, B1L.p, rt, st);
  scale_cols(rt, rk, s_lam.p, B1L.p, rt, st);
  gemm(false, true, rt, rt, rk, 1.0, B1L.p, rt, B1.p, rt, 0.0, M.p, rt, st, nullptr);
  std::vector<double> dfull(rt, 0.0);
  for (int j = 0; j < r; ++j) dfull[j] = dbar[j];
  DevBuf<double> s_df;
  upload_vec(s_df, dfull, st);
  hipLaunchKernelGGL(k_add_diag, dim3(blocks(rt)), dim3(256), 0, st, M.p, rt, s_df.p);
  symmetrize(M.p, rt, st);
  DevBuf<double> mu(std::max(rt, 1)), Sm((size_t)std::max(rt, 1) * std::max(rt, 1));
  {
    FKF_TRACE("general_addlowrank_eig", st);
    sym_eig(M.p, rt, rt, mu.p, Sm.p, rt, st, f->eig, 1e-12, f->err.p);
  }
  // the device status of this step (non-finite data, a non-positive pivot of
  // S) arrives with the eigenvalues of M
  FKF_CHECK_HIP(hipMemcpyAsync(f->err_host, f->err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  std::vector<double> muh = to_host(mu.p, rt, st);
  if (*f->err_host != 0)
    throw Error{(fkf_status)*f->err_host,
                "fkf_filter_step: the innovation covariance is not positive definite or the "
                "data are not finite"};
  const double mmax = muh.empty() ? 0.0 : muh[0];
  const double rtol = f->params.rank_rtol > 0 ? f->params.rank_rtol : 1e-14;
  const int rn = count_above(muh, rtol * mmax);
  if (rn > f->params.max_rank)
    throw Error{FKF_E_RANK, "fkf_filter_step: the low-rank term exceeds max_rank"};
  // the step succeeds: commit the state, the log-density and the new basis
  hipLaunchKernelGGL(k_add_vec, dim3(blocks(n)), dim3(256), 0, st, f->s.p, f->gdv.p, n);
  hipLaunchKernelGGL(k_add_vec, dim3(1), dim3(256), 0, st, f->ll_gen.p, f->gll.p, (int64_t)1);
  f->ll_general = true;
  // W <- [W Vh] S, Wd <- [Wd Vhd] S, D <- a1^2 mu / (1 + a1 mu)
  DevBuf<double> Wn((size_t)ldu * std::max(rn, 1)), Wdn((size_t)ldu * std::max(rn, 1));
  gemm(false, false, n, rn, rt, 1.0, Wc.p, ldu, Sm.p, rt, 0.0, Wn.p, ldu, st, nullptr);
  gemm(false, false, n, rn, rt, 1.0, Wcd.p, ldu, Sm.p, rt, 0.0, Wdn.p, ldu, st, nullptr);
  std::vector<double> dn(rn);
  for (int j = 0; j < rn; ++j) dn[j] = a1 * a1 * muh[j] / (1.0 + a1 * muh[j]);
  upload_vec(f->Dg, dn, st);
  FKF_CHECK_HIP(hipStreamSynchronize(st));
  f->W = std::move(Wn);
  f->Wd = std::move(Wdn);
  f->rg = rn;
  f->tmp.reserve(std::max(rn, 1));
  f->nu.reserve(std::max(rn, 1));
}

}  // namespace fkf

using namespace fkf;

// ========================================================== observations ===
static double obs_ll_const(const std::vector<double> &noise) {
  double s = 0.0;
  for (double r : noise) s += std::log(r);
  return -0.5 * (s + (double)noise.size() * std::log(2.0 * M_PI));
}

// Rows sorted by column with repeated columns summed (one stored entry per
// nonzero of H), so that every consumer of the operator (products with H and
// H^T, the dense H^T, the sparse moments) sees the same matrix.
static void obs_canonical(fkf_obs *o) {
  std::vector<int64_t> rp(1, 0);
  std::vector<int32_t> cl;
  std::vector<double> vl;
  cl.reserve(o->col_h.size());
  vl.reserve(o->val_h.size());
  std::vector<std::pair<int32_t, double>> row;
  int64_t mx = 0;
  for (int m = 0; m < o->n_m; ++m) {
    row.clear();
    for (int64_t e = o->rowptr_h[m]; e < o->rowptr_h[m + 1]; ++e)
      row.emplace_back(o->col_h[e], o->val_h[e]);
    std::stable_sort(row.begin(), row.end(),
                     [](const auto &a, const auto &b) { return a.first < b.first; });
    for (auto &cv : row) {
      if ((int64_t)cl.size() > rp.back() && cl.back() == cv.first) vl.back() += cv.second;
      else {
        cl.push_back(cv.first);
        vl.push_back(cv.second);
      }
    }
    rp.push_back((int64_t)cl.size());
    mx = std::max<int64_t>(mx, rp[m + 1] - rp[m]);
  }
  o->rowptr_h = std::move(rp);
  o->col_h = std::move(cl);
  o->val_h = std::move(vl);
  o->nnz = (int64_t)o->col_h.size();
  o->max_row = mx;
}

static void obs_finish(fkf_obs *o, hipStream_t st) {
  obs_canonical(o);
  o->rowptr.upload(o->rowptr_h, st);
  o->col.upload(o->col_h, st);
  o->val.upload(o->val_h, st);
  o->noise.upload(o->noise_h, st);
  if (!o->order_h.empty()) o->order.upload(o->order_h, st);
  std::vector<double> isr(o->noise_h.size());
  for (size_t i = 0; i < isr.size(); ++i) isr[i] = 1.0 / std::sqrt(o->noise_h[i]);
  o->inv_sqrt_noise.upload(isr, st);
  o->ll_const = obs_ll_const(o->noise_h);
  o->gen = g_obs_gen.fetch_add(1);
  FKF_CHECK_HIP(hipStreamSynchronize(st));
}

extern "C" fkf_status fkf_obs_create_csr(int32_t n_m, int64_t n, const int64_t *rowptr,
                                         const int32_t *col, const double *val,
                                         const double *noise_var, void *stream, fkf_obs **out) {
  return guarded([&] {
    FKF_REQUIRE(out != nullptr, "fkf_obs_create_csr: out is NULL");
    *out = nullptr;
    FKF_REQUIRE(n_m > 0 && n > 0, "fkf_obs_create_csr: sizes must be positive");
    FKF_REQUIRE(rowptr && noise_var, "fkf_obs_create_csr: NULL array");
    FKF_REQUIRE(rowptr[0] == 0, "fkf_obs_create_csr: rowptr[0] != 0");
    for (int m = 0; m < n_m; ++m)
      FKF_REQUIRE(rowptr[m + 1] >= rowptr[m], "fkf_obs_create_csr: rowptr not monotone");
    int64_t nnz = rowptr[n_m];
    FKF_REQUIRE(nnz == 0 || (col && val), "fkf_obs_create_csr: NULL col/val");
    auto o = std::make_unique<fkf_obs>();
    o->n_m = n_m;
    o->n = n;
    o->nnz = nnz;
    o->rowptr_h.assign(rowptr, rowptr + n_m + 1);
    o->col_h.assign(col, col + nnz);
    o->val_h.assign(val, val + nnz);
    for (int64_t e = 0; e < nnz; ++e) {
      FKF_REQUIRE(col[e] >= 0 && col[e] < n, "fkf_obs_create_csr: column out of range");
      FKF_REQUIRE(std::isfinite(val[e]), "fkf_obs_create_csr: non-finite value");
    }
    o->noise_h.assign(noise_var, noise_var + n_m);
    for (int m = 0; m < n_m; ++m)
      FKF_REQUIRE(noise_var[m] > 0 && std::isfinite(noise_var[m]),
                  "fkf_obs_create_csr: noise variances must be positive");
    obs_finish(o.get(), as_stream(stream));
    *out = o.release();
  });
}

extern "C" fkf_status fkf_obs_create_rays(int32_t d, const int32_t *grid, int32_t n_m,
                                          const double *src, const double *rcv,
                                          const double *noise_var, void *stream, fkf_obs **out) {
  return guarded([&] {
    FKF_REQUIRE(out != nullptr, "fkf_obs_create_rays: out is NULL");
    *out = nullptr;
    FKF_REQUIRE(grid && src && rcv && noise_var, "fkf_obs_create_rays: NULL argument");
    FKF_REQUIRE(d == 2 || d == 3, "fkf_obs_create_rays: d must be 2 or 3");
    FKF_REQUIRE(n_m > 0, "fkf_obs_create_rays: n_m must be positive");
    int64_t n = 1;
    for (int k = 0; k < d; ++k) {
      FKF_REQUIRE(grid[k] >= 1, "fkf_obs_create_rays: grid size < 1");
      n *= grid[k];
    }
    for (int64_t i = 0; i < (int64_t)n_m * d; ++i)
      FKF_REQUIRE(src[i] >= 0 && src[i] <= 1 && rcv[i] >= 0 && rcv[i] <= 1,
                  "fkf_obs_create_rays: ray endpoints must lie in the unit box");
    auto o = std::make_unique<fkf_obs>();
    trace_rays(d, grid, n_m, src, rcv, o->rowptr_h, o->col_h, o->val_h);
    {
      // Morton key of (source, receiver): 10 bits per coordinate, bits
      // interleaved from the most significant down
      std::vector<std::pair<uint64_t, int32_t>> key(n_m);
      for (int32_t m = 0; m < n_m; ++m) {
        uint32_t q[6];
        for (int k = 0; k < d; ++k) {
          q[k] = (uint32_t)std::min(1023.0, std::floor(src[(int64_t)m * d + k] * 1024.0));
          q[d + k] = (uint32_t)std::min(1023.0, std::floor(rcv[(int64_t)m * d + k] * 1024.0));
        }
        uint64_t kv = 0;
        for (int b = 9; b >= 0; --b)
          for (int k = 0; k < 2 * d; ++k) kv = (kv << 1) | ((q[k] >> b) & 1u);
        key[m] = {kv, m};
      }
      std::stable_sort(key.begin(), key.end(),
                       [](const auto &a, const auto &b) { return a.first < b.first; });
      o->order_h.resize(n_m);
      for (int32_t m = 0; m < n_m; ++m) o->order_h[m] = key[m].second;
    }
    o->n_m = n_m;
    o->n = n;
    o->nnz = (int64_t)o->col_h.size();
    o->noise_h.assign(noise_var, noise_var + n_m);
    for (int m = 0; m < n_m; ++m)
      FKF_REQUIRE(noise_var[m] > 0 && std::isfinite(noise_var[m]),
                  "fkf_obs_create_rays: noise variances must be positive");
    obs_finish(o.get(), as_stream(stream));
    *out = o.release();
  });
}

extern "C" fkf_status fkf_obs_shape(const fkf_obs *o, int32_t *n_m, int64_t *n, int64_t *nnz) {
  return guarded([&] {
    FKF_REQUIRE(o != nullptr, "fkf_obs_shape: NULL handle");
    if (n_m) *n_m = o->n_m;
    if (n) *n = o->n;
    if (nnz) *nnz = o->nnz;
  });
}

extern "C" fkf_status fkf_obs_get_csr(const fkf_obs *o, int64_t *rowptr, int32_t *col,
                                      double *val) {
  return guarded([&] {
    FKF_REQUIRE(o && rowptr && col && val, "fkf_obs_get_csr: NULL argument");
    std::copy(o->rowptr_h.begin(), o->rowptr_h.end(), rowptr);
    std::copy(o->col_h.begin(), o->col_h.end(), col);
    std::copy(o->val_h.begin(), o->val_h.end(), val);
  });
}

extern "C" fkf_status fkf_obs_apply(const fkf_obs *o, const double *x, double *y, void *stream) {
  return guarded([&] {
    FKF_REQUIRE(o && x && y, "fkf_obs_apply: NULL argument");
    spmv(o->rowptr.p, o->col.p, o->val.p, o->n_m, x, y, as_stream(stream));
    FKF_CHECK_HIP(hipGetLastError());
  });
}

extern "C" fkf_status fkf_obs_cross_cov(fkf_cov *cov, const fkf_obs *o, double *P, int64_t ldp,
                                        void *stream) {
  return guarded([&] {
    FKF_REQUIRE(cov && o && P, "fkf_obs_cross_cov: NULL argument");
    FKF_REQUIRE(cov_n(cov) == o->n, "fkf_obs_cross_cov: size mismatch between cov and obs");
    FKF_REQUIRE(ldp >= o->n, "fkf_obs_cross_cov: leading dimension < n");
    hipStream_t st = as_stream(stream);
    DevBuf<double> Ht;   // dense H^T, only where the sparse form does not apply
    cross_cov(cov, o, Ht, P, ldp, st);
    FKF_CHECK_HIP(hipStreamSynchronize(st));   // Ht is released on return
  });
}

extern "C" void fkf_obs_destroy(fkf_obs *o) {
  if (!o) return;
  (void)hipDeviceSynchronize();
  delete o;
}

// ================================================================ filter ===
extern "C" fkf_status fkf_filter_create(fkf_cov *cov, const double *s0, double alpha0,
                                        const fkf_filter_params *params, void *stream,
                                        fkf_filter **out) {
  return guarded([&] {
    FKF_REQUIRE(out != nullptr, "fkf_filter_create: out is NULL");
    *out = nullptr;
    FKF_REQUIRE(cov != nullptr, "fkf_filter_create: NULL covariance");
    FKF_REQUIRE(cov_kind(cov) < FKF_MATERN_12_DLENGTH,
                "fkf_filter_create: a length-derivative operator is not a covariance");
    FKF_REQUIRE(alpha0 >= 0 && std::isfinite(alpha0), "fkf_filter_create: alpha0 must be >= 0");
    constexpr uint32_t kParamsV1 = 16;   // struct_size of the first three fields alone
    if (params)
      FKF_REQUIRE(params->struct_size == sizeof(fkf_filter_params) ||
                      params->struct_size == kParamsV1,
                  "fkf_filter_create: params struct_size");
    hipStream_t st = as_stream(stream);
    auto f = std::make_unique<fkf_filter>();
    f->cov = cov;
    f->n = cov_n(cov);
    f->theta = cov_variance(cov);
    f->mixed = cov_mixed(cov);
    f->alpha = alpha0;
    f->params = fkf_filter_params{};
    f->params.struct_size = sizeof(fkf_filter_params);
    f->params.max_rank = 4096;
    f->params.rank_rtol = 0.0;
    f->params.gep_mode = FKF_GEP_EXACT;
    f->params.oversample = 20;
    if (params) {
      f->params.max_rank = params->max_rank;
      f->params.rank_rtol = params->rank_rtol;
      if (params->struct_size == sizeof(fkf_filter_params)) {
        FKF_REQUIRE(params->gep_mode == FKF_GEP_EXACT || params->gep_mode == FKF_GEP_RANDOMIZED,
                    "fkf_filter_create: unknown gep_mode");
        FKF_REQUIRE(params->reserved == 0, "fkf_filter_create: reserved must be 0");
        f->params.gep_mode = params->gep_mode;
        f->params.gep_rank = params->gep_rank;
        f->params.oversample = params->oversample < 0 ? 20 : params->oversample;
        f->params.seed = params->seed;
      }
    }
    f->s.alloc(f->n);
    if (s0)
      FKF_CHECK_HIP(hipMemcpyAsync(f->s.p, s0, f->n * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
      fill(f->s.p, f->n, 0.0, st);
    f->err.alloc(1);
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(1), 0, st, f->err.p, 0);
    FKF_CHECK_HIP(hipHostMalloc((void **)&f->err_host, sizeof(int)));
    *f->err_host = 0;
    FKF_CHECK_HIP(hipStreamSynchronize(st));
    *out = f.release();
  });
}

extern "C" fkf_status fkf_filter_reset(fkf_filter *f, const double *s0, double alpha0,
                                       void *stream) {
  return guarded([&] {
    FKF_REQUIRE(f != nullptr, "fkf_filter_reset: NULL handle");
    FKF_REQUIRE(alpha0 >= 0 && std::isfinite(alpha0), "fkf_filter_reset: alpha0 must be >= 0");
    hipStream_t st = as_stream(stream);
    if (s0)
      FKF_CHECK_HIP(hipMemcpyAsync(f->s.p, s0, f->n * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
      fill(f->s.p, f->n, 0.0, st);
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(1), 0, st, f->err.p, 0);
    if (f->ll_gen.p) fill(f->ll_gen.p, 1, 0.0, st);
    FKF_CHECK_HIP(hipGetLastError());
    // the device work queued before the reset may still mirror its status
    // into the pinned flag: wait for it before clearing the flag
    FKF_CHECK_HIP(hipStreamSynchronize(st));
    *f->err_host = 0;
    f->k = 0;
    f->alpha = alpha0;
    f->mode = 0;
    f->basis_gen = 0;
    f->n_m = f->nmode = 0;
    f->failed = FKF_OK;
    f->rg = 0;
    f->ll_const = 0.0;
    f->ll_general = false;
    f->lin_src = 0;
  });
}

// Argument and state checks of one filter step (throws).
static void check_step(fkf_filter *f, const fkf_obs *o, const double *y, const char *who) {
  if (!(f && o && y)) throw Error{FKF_E_ARG, std::string(who) + ": NULL argument"};
  if (f->failed != FKF_OK) throw Error{FKF_E_ORDER, std::string(who) + ": filter has failed earlier"};
  if (*f->err_host != 0) {
    f->failed = (fkf_status)*f->err_host;
    throw Error{f->failed, std::string(who) + ": a previous step produced non-finite values"};
  }
  if (o->n != f->n) throw Error{FKF_E_ARG, std::string(who) + ": operator size does not match the state"};
}

// Run the work of a step of the filters fs[0..count): an error raised after
// the argument and state checks marks every one of them failed, so that they
// refuse further steps (a failed general step leaves its filter's state as it
// was; the other failures may leave it partly updated).
template <class F>
static void step_guard(fkf_filter *const *fs, int count, F &&body) {
  try {
    body();
  } catch (const Error &e) {
    for (int i = 0; i < count; ++i)
      if (fs[i]->failed == FKF_OK) fs[i]->failed = e.code;
    throw;
  }
}

// The step after the basis (if any) is in place: prediction and update.
static void step_after_basis(fkf_filter *f, const fkf_obs *o, const double *y, hipStream_t st) {
  if (f->mode == 1 && o->gen != f->basis_gen) to_general(f, st);
  if (f->mode == 2) {
    step_general(f, o, y, st);
    FKF_CHECK_HIP(hipMemcpyAsync(f->err_host, f->err.p, sizeof(int), hipMemcpyDeviceToHost, st));
    FKF_CHECK_HIP(hipGetLastError());
    f->alpha += 1.0;
    f->k += 1;
    return;
  }
  const double alpha_new = f->alpha + 1.0;   // prediction (F = I)
  const int nm = f->n_m;
  FKF_TRACE("filter_step", st);
  hipLaunchKernelGGL(k_modes_step_eta, dim3(blocks(f->nmode, 4)), dim3(256), 0, st, f->Ve.p, nm,
                     f->nmode, y,
                     f->lam.p, f->delta.p, f->eta.p, alpha_new, f->zp.p, f->llq.p, f->err.p);
  f->ll_const += o->ll_const;
  if (f->dcov)
    hipLaunchKernelGGL(k_loglik_length_step, dim3(blocks(nm, 4)), dim3(256), 0, st, nm,
                       f->ll_Ad.p, f->ll_Cd.p, f->llq.p);
  {
    GemvEpi e;
    e.kind = kEpiAdd;
    e.err = f->err.p;
    e.err_mirror = f->err_host;
    gemv_panel(f, f->zp.p, false, f->s.p, e, st);
  }
  FKF_CHECK_HIP(hipGetLastError());
  f->alpha = alpha_new;
  f->k += 1;
}

extern "C" fkf_status fkf_filter_step(fkf_filter *f, const fkf_obs *o, const double *y,
                                      void *stream) {
  return guarded([&] {
    check_step(f, o, y, "fkf_filter_step");
    hipStream_t st = as_stream(stream);
    step_guard(&f, 1, [&] {
      if (f->mode == 0) build_basis(f, o, st);
      step_after_basis(f, o, y, st);
    });
  });
}

// The linearised operator H_k of the extended filter about the current
// estimate and the data ytil of the equivalent linear step (both held by the
// filter; the sparsity pattern is copied once per source operator).  H_k gets
// a fresh generation every step: it is a different operator each time.
static const fkf_obs *boxcox_linearize(fkf_filter *f, const fkf_obs *o, double a,
                                       const double *y, hipStream_t st) {
  if (!f->lin || f->lin_src != o->gen) {
    auto L = std::make_unique<fkf_obs>();
    L->n_m = o->n_m;
    L->n = o->n;
    L->nnz = o->nnz;
    L->max_row = o->max_row;
    L->noise_h = o->noise_h;
    L->ll_const = o->ll_const;
    L->rowptr.copy_from(o->rowptr.p, (size_t)o->n_m + 1, st);
    L->col.copy_from(o->col.p, (size_t)o->nnz, st);
    L->noise.copy_from(o->noise.p, (size_t)o->n_m, st);
    L->inv_sqrt_noise.copy_from(o->inv_sqrt_noise.p, (size_t)o->n_m, st);
    L->val.alloc((size_t)o->nnz);
    f->lin = std::move(L);
    f->lin_src = o->gen;
  }
  f->ytil.reserve((size_t)o->n_m);
  hipLaunchKernelGGL(k_boxcox_linearize, dim3(blocks(o->n_m, 4)), dim3(256), 0, st, o->rowptr.p,
                     o->col.p, o->val.p, o->n_m, f->s.p, a, y, f->lin->val.p, f->ytil.p,
                     f->err.p);
  FKF_CHECK_HIP(hipGetLastError());
  f->lin->gen = g_obs_gen.fetch_add(1);
  return f->lin.get();
}

extern "C" fkf_status fkf_filter_step_boxcox(fkf_filter *f, const fkf_obs *o, double bc_alpha,
                                             const double *y, void *stream) {
  return guarded([&] {
    check_step(f, o, y, "fkf_filter_step_boxcox");
    FKF_REQUIRE(std::isfinite(bc_alpha) && bc_alpha > 0,
                "fkf_filter_step_boxcox: bc_alpha must be finite and positive");
    hipStream_t st = as_stream(stream);
    step_guard(&f, 1, [&] {
      const fkf_obs *lin;
      {
        FKF_TRACE("boxcox_linearize", st);
        lin = boxcox_linearize(f, o, bc_alpha, y, st);
      }
      if (f->mode == 0) build_basis(f, lin, st);
      step_after_basis(f, lin, f->ytil.p, st);
    });
  });
}

extern "C" fkf_status fkf_filter_step_many(fkf_filter *const *filters, const fkf_obs *const *obs,
                                           const double *const *y, int32_t count, void *stream) {
  return guarded([&] {
    FKF_REQUIRE(count >= 0, "fkf_filter_step_many: count < 0");
    if (count == 0) return;
    FKF_REQUIRE(filters && obs && y, "fkf_filter_step_many: NULL array");
    for (int i = 0; i < count; ++i) {
      check_step(filters[i], obs[i], y[i], "fkf_filter_step_many");
      for (int j = 0; j < i; ++j)
        FKF_REQUIRE(filters[j] != filters[i], "fkf_filter_step_many: a filter appears twice");
    }
    hipStream_t st = as_stream(stream);
    step_guard(filters, count, [&] {
      std::vector<fkf_filter *> nf;
      std::vector<const fkf_obs *> no;
      for (int i = 0; i < count; ++i)
        if (filters[i]->mode == 0) {
          if (filters[i]->params.gep_mode == FKF_GEP_RANDOMIZED) {
            build_basis_randomized(filters[i], obs[i], st);
            continue;
          }
          nf.push_back(filters[i]);
          no.push_back(obs[i]);
        }
      if (!nf.empty()) build_bases(nf.data(), no.data(), (int)nf.size(), st);
      if (count == 1) {
        step_after_basis(filters[0], obs[0], y[0], st);
        return;
      }
      // the steps of independent filters run on the stream lanes
      LanePool &lp = lane_pool();
      const std::vector<int> lane = lanes_of(filters, count);
      lanes_fork(lp, st);
      for (int i = 0; i < count; ++i) step_after_basis(filters[i], obs[i], y[i], lp.s[lane[i]]);
      lanes_join(lp, st);
    });
  });
}

extern "C" fkf_status fkf_filter_status(fkf_filter *f, void *stream) {
  fkf_status inner = FKF_OK;
  fkf_status rc = guarded([&] {
    FKF_REQUIRE(f != nullptr, "fkf_filter_status: NULL handle");
    hipStream_t st = as_stream(stream);
    int e = 0;
    FKF_CHECK_HIP(hipMemcpyAsync(&e, f->err.p, sizeof(int), hipMemcpyDeviceToHost, st));
    FKF_CHECK_HIP(hipStreamSynchronize(st));
    if (e != 0 && f->failed == FKF_OK) f->failed = (fkf_status)e;
    inner = f->failed;
    if (inner != FKF_OK) set_error("filter latched a device-side failure");
  });
  return rc != FKF_OK ? rc : inner;
}

extern "C" fkf_status fkf_filter_mean(const fkf_filter *f, double *s_dev, void *stream) {
  return guarded([&] {
    FKF_REQUIRE(f && s_dev, "fkf_filter_mean: NULL argument");
    FKF_CHECK_HIP(hipMemcpyAsync(s_dev, f->s.p, f->n * sizeof(double), hipMemcpyDeviceToDevice,
                                 as_stream(stream)));
  });
}

extern "C" fkf_status fkf_filter_variance(const fkf_filter *f, double *var, void *stream) {
  return guarded([&] {
    FKF_REQUIRE(f && var, "fkf_filter_variance: NULL argument");
    hipStream_t st = as_stream(stream);
    const double base = f->alpha * f->theta;   // alpha_k diag(Gamma), Matern diag = theta
    if (f->mode == 0) {
      fill(var, f->n, base, st);
      return;
    }
    fkf_filter *mf = const_cast<fkf_filter *>(f);
    GemvEpi e;
    e.kind = kEpiVar;
    e.base = base;
    if (f->mode == 2) {
      if (f->rg == 0) fill(var, f->n, base, st);
      else gemv_panel_m(f->W.p, f->ldu, f->rg, f->n, f->Dg.p, true, var, e, st);
      FKF_CHECK_HIP(hipGetLastError());
      return;
    }
    gemv_panel(mf, f->delta.p, true, var, e, st);
    FKF_CHECK_HIP(hipGetLastError());
  });
}

extern "C" fkf_status fkf_filter_realize(const fkf_filter *f, const double *g, int32_t ns,
                                         int64_t ldg, double *out, int64_t ldo, void *stream) {
  return guarded([&] {
    FKF_REQUIRE(f != nullptr, "fkf_filter_realize: NULL handle");
    FKF_REQUIRE(ns >= 0, "fkf_filter_realize: ns < 0");
    if (ns == 0) return;
    FKF_REQUIRE(g && out, "fkf_filter_realize: NULL array");
    FKF_REQUIRE(ldg >= f->n && ldo >= f->n, "fkf_filter_realize: leading dimension < n");
    hipStream_t st = as_stream(stream);
    fkf_filter *mf = const_cast<fkf_filter *>(f);
    const double sa = std::sqrt(f->alpha);
    for (int c = 0; c < ns; ++c) {
      const double *gc = g + ldg * c;
      double *oc = out + ldo * c;
      if (f->mode == 0 || f->alpha == 0.0 || (f->mode == 2 && f->rg == 0)) {
        // no low-rank term: Sigma = alpha Gamma and the realization is s + alpha^1/2 g
        hipLaunchKernelGGL(k_axpy_out, dim3(blocks(f->n)), dim3(256), 0, st, f->s.p, gc, sa, oc,
                           f->n);
        continue;
      }
      if (f->mode == 2) {
        // zz = Sigma_- (Wd^T g); out = s + a^1/2 (g - W zz)
        gemm(true, false, f->rg, 1, f->n, 1.0, f->Wd.p, f->ldu, gc, f->n, 0.0, mf->nu.p, f->rg, st,
             &mf->gwork);
        hipLaunchKernelGGL(k_sigma_minus, dim3(blocks(f->rg)), dim3(256), 0, st, f->Dg.p, f->nu.p,
                           f->rg, f->alpha, mf->tmp.p);
        GemvEpi e;
        e.kind = kEpiRealize;
        e.s = f->s.p;
        e.g = gc;
        e.salpha = sa;
        gemv_panel_m(f->W.p, f->ldu, f->rg, f->n, f->tmp.p, false, oc, e, st);
        continue;
      }
      // h = H g with the basis' operator; zz = (Sigma_- / lambda) Ve^T h; out = s + a^1/2 (g - U0 zz)
      hipLaunchKernelGGL(k_spmv_f, dim3(blocks(f->n_m, 4)), dim3(256), 0, st, f->b_rowptr.p,
                         f->b_col.p, f->b_val.p, f->n_m, gc, mf->nu.p);
      hipLaunchKernelGGL(k_modes_realize, dim3(blocks(f->nmode, 4)), dim3(256), 0, st, f->Ve.p,
                         f->n_m, f->nmode, f->nu.p, f->lam.p, f->delta.p, f->alpha, mf->tmp.p);
      GemvEpi e;
      e.kind = kEpiRealize;
      e.s = f->s.p;
      e.g = gc;
      e.salpha = sa;
      gemv_panel(mf, f->tmp.p, false, oc, e, st);
    }
    FKF_CHECK_HIP(hipGetLastError());
  });
}

extern "C" fkf_status fkf_gaussian_sketch(uint64_t seed, int64_t count, double *out,
                                          void *stream) {
  return guarded([&] {
    FKF_REQUIRE(count >= 0, "fkf_gaussian_sketch: count < 0");
    if (count == 0) return;
    FKF_REQUIRE(out != nullptr, "fkf_gaussian_sketch: NULL array");
    hipLaunchKernelGGL(k_sketch_normals, dim3(blocks((count + 1) / 2)), dim3(256), 0,
                       as_stream(stream), seed, count, out);
    FKF_CHECK_HIP(hipGetLastError());
  });
}

extern "C" fkf_status fkf_filter_info(const fkf_filter *f, int64_t *k, double *alpha,
                                      int32_t *rank) {
  return guarded([&] {
    FKF_REQUIRE(f != nullptr, "fkf_filter_info: NULL handle");
    if (k) *k = f->k;
    if (alpha) *alpha = f->alpha;
    if (rank) *rank = f->mode == 0 ? 0 : (f->mode == 1 ? f->nmode : f->rg);
  });
}

extern "C" fkf_status fkf_filter_track_length(fkf_filter *f, fkf_cov *dcov, void *stream) {
  (void)stream;
  return guarded([&] {
    FKF_REQUIRE(f && dcov, "fkf_filter_track_length: NULL argument");
    if (f->mode != 0 || f->k != 0)
      throw Error{FKF_E_ORDER, "fkf_filter_track_length: must be called before the first step"};
    FKF_REQUIRE(cov_kind(dcov) == cov_kind(f->cov) + FKF_MATERN_12_DLENGTH,
                "fkf_filter_track_length: dcov must be the length derivative of the filter's kernel");
    FKF_REQUIRE(cov_n(dcov) == f->n, "fkf_filter_track_length: size mismatch");
    if (f->params.gep_mode != FKF_GEP_EXACT)
      throw Error{FKF_E_UNSUPPORTED,
                  "fkf_filter_track_length: the length derivative needs the exact eigensolver"};
    FKF_REQUIRE(cov_length(dcov) == cov_length(f->cov),
                "fkf_filter_track_length: length differs from the filter's covariance");
    f->dcov = dcov;
  });
}

extern "C" fkf_status fkf_filter_loglik(const fkf_filter *f, double *ll, double *dll_dlog_theta,
                                        double *dll_dlog_length, double *dll_dlog_noise,
                                        void *stream) {
  return guarded([&] {
    FKF_REQUIRE(f && ll, "fkf_filter_loglik: NULL argument");
    if (f->mode == 1 && f->nmode < f->n_m)
      throw Error{FKF_E_UNSUPPORTED, "fkf_filter_loglik: the constant-H basis keeps fewer modes "
                                     "than measurements (truncated randomized eigensolver)"};
    if ((dll_dlog_theta || dll_dlog_length || dll_dlog_noise) && f->ll_general)
      throw Error{FKF_E_UNSUPPORTED,
                  "fkf_filter_loglik: derivatives are available while every step is a constant-H "
                  "step"};
    if (dll_dlog_length && !f->dcov)
      throw Error{FKF_E_ORDER, "fkf_filter_loglik: length derivative not tracked "
                               "(fkf_filter_track_length before the first step)"};
    hipStream_t st = as_stream(stream);
    double tot = f->ll_const, ga = 0.0, gl = 0.0, gs = 0.0;
    if (f->llq.p) {
      const std::vector<double> q = to_host(f->llq.p, (size_t)kLLStride * f->nmode, st);
      for (size_t j = 0; j + kLLStride <= q.size(); j += kLLStride) {
        tot += q[j + 4];
        ga += q[j + 5];
        gs += q[j + 6];
        gl += q[j + 9];
      }
    }
    if (f->ll_gen.p) tot += to_host(f->ll_gen.p, 1, st)[0];
    *ll = tot;
    if (dll_dlog_theta) *dll_dlog_theta = ga;
    if (dll_dlog_length) *dll_dlog_length = f->dcov ? gl * cov_length(f->cov) : 0.0;
    if (dll_dlog_noise) *dll_dlog_noise = gs;
  });
}

extern "C" fkf_status fkf_filter_modes(const fkf_filter *f, double *lam_host, double *w_host) {
  return guarded([&] {
    FKF_REQUIRE(f && lam_host && w_host, "fkf_filter_modes: NULL argument");
    if (f->mode != 1) throw Error{FKF_E_ORDER, "fkf_filter_modes: no constant-H basis"};
    std::vector<double> lam(f->nmode), del(f->nmode);
    FKF_CHECK_HIP(hipDeviceSynchronize());
    FKF_CHECK_HIP(hipMemcpy(lam.data(), f->lam.p, f->nmode * sizeof(double), hipMemcpyDeviceToHost));
    FKF_CHECK_HIP(hipMemcpy(del.data(), f->delta.p, f->nmode * sizeof(double), hipMemcpyDeviceToHost));
    for (int j = 0; j < f->nmode; ++j) {
      lam_host[j] = lam[j];
      w_host[j] = f->alpha - del[j] * lam[j];
    }
  });
}

extern "C" fkf_status fkf_filter_lowrank(const fkf_filter *f, double *W_dev, int64_t ldw,
                                         double *Wd_dev, int64_t ldwd, double *D_dev,
                                         int32_t capacity, int32_t *rank, void *stream) {
  return guarded([&] {
    FKF_REQUIRE(f && rank, "fkf_filter_lowrank: NULL argument");
    FKF_REQUIRE(ldw >= f->n && ldwd >= f->n, "fkf_filter_lowrank: leading dimension < n");
    hipStream_t st = as_stream(stream);
    const int64_t n = f->n;
    *rank = 0;
    if (f->mode == 0) return;
    if (f->mode == 2) {
      const int r = f->rg;
      FKF_REQUIRE(capacity >= r, "fkf_filter_lowrank: capacity below the rank");
      if (W_dev) copy2d(n, r, f->W.p, f->ldu, W_dev, ldw, st);
      if (Wd_dev) copy2d(n, r, f->Wd.p, f->ldu, Wd_dev, ldwd, st);
      if (D_dev && r)
        FKF_CHECK_HIP(hipMemcpyAsync(D_dev, f->Dg.p, r * sizeof(double), hipMemcpyDeviceToDevice, st));
      FKF_CHECK_HIP(hipStreamSynchronize(st));
      *rank = r;
      return;
    }
    // constant-H form: W = U0 Lambda^-1/2, Wd = H_b^T Ve Lambda^-1/2, D = delta lambda over
    // the modes with lambda > 1e-13 lambda_max (as the change to the general form)
    const int nm = f->n_m;
    FKF_REQUIRE(capacity >= f->nmode, "fkf_filter_lowrank: capacity below the rank");
    std::vector<double> lam = to_host(f->lam.p, f->nmode, st),
                        del = to_host(f->delta.p, f->nmode, st);
    const int r = count_above(lam, 1e-13 * (lam.empty() ? 0.0 : lam[0]));
    std::vector<double> isl(r), dg(r);
    for (int j = 0; j < r; ++j) {
      isl[j] = 1.0 / std::sqrt(lam[j]);
      dg[j] = del[j] * lam[j];
    }
    DevBuf<double> s_isl;
    upload_vec(s_isl, isl, st);
    if (W_dev && r) {
      copy2d(n, r, f->U0.p, f->ldu, W_dev, ldw, st);
      scale_cols(n, r, s_isl.p, W_dev, ldw, st);
    }
    if (Wd_dev && r) {
      DevBuf<double> Hbt((size_t)n * nm);
      dense_ht(f->b_rowptr.p, f->b_col.p, f->b_val.p, nm, n, Hbt.p, st);
      gemm(false, false, n, r, nm, 1.0, Hbt.p, n, f->Ve.p, nm, 0.0, Wd_dev, ldwd, st, nullptr);
      scale_cols(n, r, s_isl.p, Wd_dev, ldwd, st);
      FKF_CHECK_HIP(hipStreamSynchronize(st));   // Hbt is released on return
    }
    if (D_dev && r)
      FKF_CHECK_HIP(hipMemcpyAsync(D_dev, dg.data(), r * sizeof(double), hipMemcpyHostToDevice, st));
    FKF_CHECK_HIP(hipStreamSynchronize(st));
    *rank = r;
  });
}

extern "C" void fkf_filter_destroy(fkf_filter *f) {
  if (!f) return;
  (void)hipDeviceSynchronize();
  delete f;
}
