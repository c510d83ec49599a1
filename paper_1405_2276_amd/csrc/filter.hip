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
#include <algorithm>
#include <atomic>
#include <cmath>
#include <memory>

#include "kernels.h"
#include "linalg.h"
#include "trace.h"

struct fkf_obs {
  int n_m = 0;
  int64_t n = 0, nnz = 0;
  uint64_t gen = 0;
  std::vector<int64_t> rowptr_h;
  std::vector<int32_t> col_h;
  std::vector<double> val_h, noise_h;
  fkf::DevBuf<int64_t> rowptr;
  fkf::DevBuf<int32_t> col;
  fkf::DevBuf<double> val, noise, inv_sqrt_noise;
};

struct fkf_filter {
  fkf_cov *cov = nullptr;
  int64_t n = 0, ldu = 0;
  double theta = 1.0;
  fkf_filter_params params{};
  int64_t k = 0;
  double alpha = 0.0;
  int mode = 0;            // 0: no low-rank term yet, 1: constant-H basis
  uint64_t basis_gen = 0;
  int n_m = 0;
  fkf_status failed = FKF_OK;
  fkf::DevBuf<double> s, U0, Ve, lam, delta, nu, zp, part, tmp;
  fkf::DevBuf<int64_t> b_rowptr;   // copy of the basis' measurement operator
  fkf::DevBuf<int32_t> b_col;
  fkf::DevBuf<double> b_val;
  fkf::DevBuf<int> err;
  int *err_host = nullptr;
  fkf::EigWork eig;
  ~fkf_filter() {
    if (err_host) (void)hipHostFree(err_host);
  }
};

namespace fkf {

// implemented in hmat.hip
double cov_variance(const fkf_cov *cov);
int64_t cov_n(const fkf_cov *cov);

static std::atomic<uint64_t> g_obs_gen{1};

constexpr int kSegCols = 32;    // columns per GEMV workgroup
constexpr int kRowsPerWG = 512; // 256 threads x 2 rows

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

// One wavefront per mode j: z_j = Ve[:, j] . nu, then the per-mode update.
__global__ void __launch_bounds__(256) k_modes_step(const double *__restrict__ Ve, int n_m,
                                                    const double *__restrict__ nu,
                                                    const double *__restrict__ lam,
                                                    double *__restrict__ delta, double alpha,
                                                    double *__restrict__ zp, int *err) {
  int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n_m) return;
  int l = threadIdx.x & 63;
  const double *v = Ve + (int64_t)n_m * j;
  double z = 0;
  for (int m = l; m < n_m; m += 64) z = fma(v[m], nu[m], z);
  z = wave_sum(z);
  if (l == 0) {
    double lj = lam[j], dj = delta[j];
    double a = alpha - dj * lj;          // alpha_{k+1} - D_k
    double den = 1.0 + a * lj;           // (alpha - D) lambda + 1: S_k in the eigenbasis
    double g = a / den;
    zp[j] = g * z;
    delta[j] = dj + a * g;               // D_{k+1} / lambda
    if (!isfinite(zp[j]) || !isfinite(delta[j])) atomicExch(err, (int)FKF_E_NONFINITE);
  }
}

// One wavefront per mode j: realization coefficients
// zz_j = (Ve[:, j] . h) * Sigma_-_j / lambda_j with Sigma_- = 1 - (1 - D/alpha)^1/2,
// written as (delta/alpha) / (1 + (1 - delta lambda / alpha)^1/2).
__global__ void __launch_bounds__(256) k_modes_realize(const double *__restrict__ Ve, int n_m,
                                                       const double *__restrict__ h,
                                                       const double *__restrict__ lam,
                                                       const double *__restrict__ delta,
                                                       double alpha, double *__restrict__ zz) {
  int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n_m) return;
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

// Segmented tall GEMV: part[seg][i] = sum_{j in seg} f(U0[i, j]) z[j] with
// f(u) = u (SQUARE = false) or u^2 (SQUARE = true).  Two rows per thread with
// 16-byte loads; every workgroup streams kSegCols columns of a 512-row panel.
template <bool SQUARE>
__global__ void __launch_bounds__(256) k_gemv_seg(const double *__restrict__ U0, int64_t n,
                                                  int64_t ldu, int n_m,
                                                  const double *__restrict__ z,
                                                  double *__restrict__ part) {
  int64_t i0 = (int64_t)blockIdx.x * kRowsPerWG + 2 * threadIdx.x;
  int j0 = blockIdx.y * kSegCols;
  int jn = min(kSegCols, n_m - j0);
  if (i0 >= n) return;
  double a0 = 0, a1 = 0;
  const v2d *src = reinterpret_cast<const v2d *>(U0 + i0 + ldu * j0);
  const int64_t ld2 = ldu / 2;
  if (jn == kSegCols) {
    v2d u[kSegCols];
#pragma unroll
    for (int jj = 0; jj < kSegCols; ++jj) u[jj] = __builtin_nontemporal_load(src + ld2 * jj);
#pragma unroll
    for (int jj = 0; jj < kSegCols; ++jj) {
      double zj = z[j0 + jj];
      if (SQUARE) {
        a0 = fma(u[jj].x * u[jj].x, zj, a0);
        a1 = fma(u[jj].y * u[jj].y, zj, a1);
      } else {
        a0 = fma(u[jj].x, zj, a0);
        a1 = fma(u[jj].y, zj, a1);
      }
    }
  } else {
    for (int jj = 0; jj < jn; ++jj) {
      v2d u = src[ld2 * jj];
      double zj = z[j0 + jj];
      if (SQUARE) {
        a0 = fma(u.x * u.x, zj, a0);
        a1 = fma(u.y * u.y, zj, a1);
      } else {
        a0 = fma(u.x, zj, a0);
        a1 = fma(u.y, zj, a1);
      }
    }
  }
  double *o = part + (int64_t)blockIdx.y * n;
  o[i0] = a0;
  if (i0 + 1 < n) o[i0 + 1] = a1;
}

// s[i] += sum_seg part[seg][i]
__global__ void k_seg_add(const double *__restrict__ part, int nseg, int64_t n,
                          double *__restrict__ s) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0;
  for (int g = 0; g < nseg; ++g) a += part[(int64_t)g * n + i];
  s[i] += a;
}

// var[i] = alpha theta - sum_seg part[seg][i]
__global__ void k_seg_var(const double *__restrict__ part, int nseg, int64_t n, double base,
                          double *__restrict__ var) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0;
  for (int g = 0; g < nseg; ++g) a += part[(int64_t)g * n + i];
  var[i] = base - a;
}

// out[i] = s[i] + sqrt(alpha) (g[i] - sum_seg part[seg][i])
__global__ void k_seg_realize(const double *__restrict__ part, int nseg, int64_t n,
                              const double *__restrict__ s, const double *__restrict__ g,
                              double salpha, double *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0;
  for (int q = 0; q < nseg; ++q) a += part[(int64_t)q * n + i];
  out[i] = s[i] + salpha * (g[i] - a);
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

__global__ void k_set_flag(int *p, int v) { *p = v; }

__global__ void k_clamp_nonneg(double *__restrict__ x, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(x[i] > 0.0)) x[i] = 0.0;
}

__global__ void k_copy_strided(const double *__restrict__ src, double *__restrict__ dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// --------------------------------------------------------------- helpers ---
static unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

static void gemv_seg(const fkf_filter *f, const double *z, bool square, hipStream_t st) {
  FKF_TRACE(square ? "filter_gemv_sq" : "filter_gemv", st);
  int nseg = (f->n_m + kSegCols - 1) / kSegCols;
  dim3 grid(blocks(f->n, kRowsPerWG), (unsigned)nseg);
  if (square)
    hipLaunchKernelGGL(k_gemv_seg<true>, grid, dim3(256), 0, st, f->U0.p, f->n, f->ldu, f->n_m, z,
                       f->part.p);
  else
    hipLaunchKernelGGL(k_gemv_seg<false>, grid, dim3(256), 0, st, f->U0.p, f->n, f->ldu, f->n_m, z,
                       f->part.p);
}

// Generalized eigenpairs of H^T R^-1 H against Gamma^-1 by Rayleigh-Ritz on
// range(Gamma H^T), and the constant-H basis U0 = P Ve.
static void build_basis(fkf_filter *f, const fkf_obs *o, hipStream_t st) {
  FKF_TRACE("gep_total", st);
  const int64_t n = f->n;
  const int nm = o->n_m;
  DevBuf<double> Ht((size_t)n * nm), P((size_t)n * nm);
  dense_ht(o->rowptr.p, o->col.p, o->val.p, nm, n, Ht.p, st);
  fkf_status rc;
  {
    FKF_TRACE("gep_cross_cov", st);
    rc = fkf_cov_apply(f->cov, Ht.p, n, nm, P.p, n, (void *)st);
  }
  if (rc != FKF_OK) throw Error{rc, std::string("covariance product failed: ") + fkf_last_error()};
  Ht.release();
  DevBuf<double> G((size_t)nm * nm), A((size_t)nm * nm);
  innovation_gram(o->rowptr.p, o->col.p, o->val.p, nm, n, P.p, o->noise.p, G.p, A.p, st);
  f->lam.alloc(nm);
  f->Ve.alloc((size_t)nm * nm);
  {
    FKF_TRACE("gep_eig", st);
    sym_eig(A.p, nm, nm, f->lam.p, f->Ve.p, nm, st, f->eig);
  }
  hipLaunchKernelGGL(k_clamp_nonneg, dim3(blocks(nm)), dim3(256), 0, st, f->lam.p, nm);
  scale_rows(nm, nm, o->inv_sqrt_noise.p, f->Ve.p, nm, st);
  f->ldu = (n + 63) / 64 * 64;
  f->U0.alloc((size_t)f->ldu * nm);
  fill(f->U0.p, f->ldu * nm, 0.0, st);
  {
    FKF_TRACE("gep_basis_gemm", st);
    gemm_nn(n, nm, nm, P.p, n, f->Ve.p, nm, f->U0.p, f->ldu, st);
  }
  f->delta.alloc(nm);
  fill(f->delta.p, nm, 0.0, st);
  f->nu.alloc(nm);
  f->zp.alloc(nm);
  f->tmp.alloc(nm);
  int nseg = (nm + kSegCols - 1) / kSegCols;
  f->part.alloc((size_t)nseg * n);
  f->b_rowptr.upload(o->rowptr_h, st);
  f->b_col.upload(o->col_h, st);
  f->b_val.upload(o->val_h, st);
  f->n_m = nm;
  f->mode = 1;
  f->basis_gen = o->gen;
  FKF_CHECK_HIP(hipStreamSynchronize(st));   // P, Ht, G, A are released on return
}

}  // namespace fkf

using namespace fkf;

// ========================================================== observations ===
static void obs_finish(fkf_obs *o, hipStream_t st) {
  o->rowptr.upload(o->rowptr_h, st);
  o->col.upload(o->col_h, st);
  o->val.upload(o->val_h, st);
  o->noise.upload(o->noise_h, st);
  std::vector<double> isr(o->noise_h.size());
  for (size_t i = 0; i < isr.size(); ++i) isr[i] = 1.0 / std::sqrt(o->noise_h[i]);
  o->inv_sqrt_noise.upload(isr, st);
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
    FKF_REQUIRE(alpha0 >= 0 && std::isfinite(alpha0), "fkf_filter_create: alpha0 must be >= 0");
    if (params) FKF_REQUIRE(params->struct_size == sizeof(fkf_filter_params),
                            "fkf_filter_create: params struct_size");
    hipStream_t st = as_stream(stream);
    auto f = std::make_unique<fkf_filter>();
    f->cov = cov;
    f->n = cov_n(cov);
    f->theta = cov_variance(cov);
    f->alpha = alpha0;
    if (params) {
      f->params = *params;
    } else {
      f->params.struct_size = sizeof(fkf_filter_params);
      f->params.max_rank = 4096;
      f->params.rank_rtol = 0.0;
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

extern "C" fkf_status fkf_filter_step(fkf_filter *f, const fkf_obs *o, const double *y,
                                      void *stream) {
  return guarded([&] {
    FKF_REQUIRE(f && o && y, "fkf_filter_step: NULL argument");
    if (f->failed != FKF_OK) throw Error{FKF_E_ORDER, "fkf_filter_step: filter has failed earlier"};
    if (*f->err_host != 0) {
      f->failed = (fkf_status)*f->err_host;
      throw Error{f->failed, "fkf_filter_step: a previous step produced non-finite values"};
    }
    FKF_REQUIRE(o->n == f->n, "fkf_filter_step: operator size does not match the state");
    hipStream_t st = as_stream(stream);
    if (f->mode == 0) {
      build_basis(f, o, st);
    } else if (o->gen != f->basis_gen) {
      throw Error{FKF_E_UNSUPPORTED, "fkf_filter_step: a new measurement operator after the "
                                     "first step needs the general update"};
    }
    const double alpha_new = f->alpha + 1.0;   // prediction (F = I)
    const int nm = f->n_m;
    FKF_TRACE("filter_step", st);
    hipLaunchKernelGGL(k_innov, dim3(blocks(nm, 4), 1), dim3(256), 0, st, o->rowptr.p, o->col.p,
                       o->val.p, nm, f->s.p, y, f->nu.p, f->err.p);
    hipLaunchKernelGGL(k_modes_step, dim3(blocks(nm, 4)), dim3(256), 0, st, f->Ve.p, nm, f->nu.p,
                       f->lam.p, f->delta.p, alpha_new, f->zp.p, f->err.p);
    gemv_seg(f, f->zp.p, false, st);
    int nseg = (nm + kSegCols - 1) / kSegCols;
    hipLaunchKernelGGL(k_seg_add, dim3(blocks(f->n)), dim3(256), 0, st, f->part.p, nseg, f->n,
                       f->s.p);
    FKF_CHECK_HIP(hipMemcpyAsync(f->err_host, f->err.p, sizeof(int), hipMemcpyDeviceToHost, st));
    FKF_CHECK_HIP(hipGetLastError());
    f->alpha = alpha_new;
    f->k += 1;
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
    gemv_seg(mf, f->delta.p, true, st);
    int nseg = (f->n_m + kSegCols - 1) / kSegCols;
    hipLaunchKernelGGL(k_seg_var, dim3(blocks(f->n)), dim3(256), 0, st, f->part.p, nseg, f->n, base,
                       var);
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
    int nseg = (f->n_m + kSegCols - 1) / kSegCols;
    for (int c = 0; c < ns; ++c) {
      const double *gc = g + ldg * c;
      double *oc = out + ldo * c;
      if (f->mode == 0 || f->alpha == 0.0) {
        // no low-rank term: Sigma = alpha Gamma and the realization is s + alpha^1/2 g
        hipLaunchKernelGGL(k_axpy_out, dim3(blocks(f->n)), dim3(256), 0, st, f->s.p, gc, sa, oc,
                           f->n);
        continue;
      }
      // h = H g with the basis' operator; zz = (Sigma_- / lambda) Ve^T h; out = s + a^1/2 (g - U0 zz)
      hipLaunchKernelGGL(k_spmv_f, dim3(blocks(f->n_m, 4)), dim3(256), 0, st, f->b_rowptr.p,
                         f->b_col.p, f->b_val.p, f->n_m, gc, mf->nu.p);
      hipLaunchKernelGGL(k_modes_realize, dim3(blocks(f->n_m, 4)), dim3(256), 0, st, f->Ve.p,
                         f->n_m, f->nu.p, f->lam.p, f->delta.p, f->alpha, mf->tmp.p);
      gemv_seg(mf, f->tmp.p, false, st);
      hipLaunchKernelGGL(k_seg_realize, dim3(blocks(f->n)), dim3(256), 0, st, f->part.p, nseg, f->n,
                         f->s.p, gc, sa, oc);
    }
    FKF_CHECK_HIP(hipGetLastError());
  });
}

extern "C" fkf_status fkf_filter_info(const fkf_filter *f, int64_t *k, double *alpha,
                                      int32_t *rank) {
  return guarded([&] {
    FKF_REQUIRE(f != nullptr, "fkf_filter_info: NULL handle");
    if (k) *k = f->k;
    if (alpha) *alpha = f->alpha;
    if (rank) *rank = f->mode == 0 ? 0 : f->n_m;
  });
}

extern "C" fkf_status fkf_filter_modes(const fkf_filter *f, double *lam_host, double *w_host) {
  return guarded([&] {
    FKF_REQUIRE(f && lam_host && w_host, "fkf_filter_modes: NULL argument");
    if (f->mode != 1) throw Error{FKF_E_ORDER, "fkf_filter_modes: no constant-H basis"};
    std::vector<double> lam(f->n_m), del(f->n_m);
    FKF_CHECK_HIP(hipDeviceSynchronize());
    FKF_CHECK_HIP(hipMemcpy(lam.data(), f->lam.p, f->n_m * sizeof(double), hipMemcpyDeviceToHost));
    FKF_CHECK_HIP(hipMemcpy(del.data(), f->delta.p, f->n_m * sizeof(double), hipMemcpyDeviceToHost));
    for (int j = 0; j < f->n_m; ++j) {
      lam_host[j] = lam[j];
      w_host[j] = f->alpha - del[j] * lam[j];
    }
  });
}

extern "C" void fkf_filter_destroy(fkf_filter *f) {
  if (!f) return;
  (void)hipDeviceSynchronize();
  delete f;
}
