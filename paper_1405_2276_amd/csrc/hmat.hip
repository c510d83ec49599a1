// Gamma_sys as a hierarchical matrix on the GPU: build (near-field assembly)
// and application Y = Gamma X (Section 2.2.1).
//
// Layout in HBM
//   * points: d x N structure-of-arrays, in cluster-tree order.
//   * near field: the symmetric half of the inadmissible leaf pairs (s <= t),
//     each a 64 x 64 FP64 tile (zero padded for a ragged leaf) stored in
//     "lane-slice" order: slice k (1 KiB) holds, for each of the 64 lanes of a
//     wavefront, two consecutive entries of that lane's 8 x 8 sub-tile, so one
//     wave-wide 16-byte load reads 1 KiB contiguously.
//   * far field: admissible blocks Gamma_st ~ U_s K(xi_s, xi_t) U_t^T with
//     tensor Chebyshev interpolation.  Neither U nor K is stored: U is
//     evaluated from the point coordinates and K from the node coordinates
//     inside the kernels, so the far field costs no HBM bytes beyond its
//     coefficient vectors.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>

#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace fkf {

struct FarCluster {
  int64_t begin, end;
  int64_t coef_off;   // offset (in units of coefficients) of this cluster
  int32_t p, pd;      // nodes per dimension, p^d
  double ctr[kMaxDim], hw[kMaxDim];
};

}  // namespace fkf

struct fkf_cov {
  int64_t n = 0;
  int d = 2;
  int kind = 0;
  double theta = 1, ell = 1;
  fkf_hmat_params hp{};
  fkf::Tree tree;
  std::vector<int> level_p;
  int n_leaves = 0;
  int64_t n_blk = 0, n_near_pairs = 0, n_far_pairs = 0, n_coef = 0, covered = 0;
  int n_fc = 0;
  int max_pd = 1;
  fkf::DevBuf<int64_t> perm;
  fkf::DevBuf<double> pts;          // d x n, tree order
  fkf::DevBuf<int64_t> leaf_off;    // n_leaves + 1
  fkf::DevBuf<int32_t> blk_s, blk_t;
  fkf::DevBuf<double> blk;          // n_blk x 4096
  fkf::DevBuf<int32_t> part_ptr, part_idx;   // per leaf: entries blk*2 + side
  fkf::DevBuf<int32_t> near_ptr, near_idx;   // per leaf: entries blk*2 + transposed
  fkf::DevBuf<fkf::FarCluster> fc;
  fkf::DevBuf<int32_t> far_ptr, far_col;     // partners per target far cluster
  fkf::DevBuf<int32_t> anc_ptr, anc_idx;     // far-cluster ancestors of each leaf
  fkf::DevBuf<double> cheb;                  // [p][a] nodes and weights
  // workspace
  fkf::DevBuf<double> xt, yt, part, xhat, yhat;
};

namespace fkf {

// ------------------------------------------------------------ device code ---
__device__ __forceinline__ double matern_dev(double r, int kind, double inv_ell, double theta) {
  if (kind == FKF_MATERN_12) return theta * exp(-r * inv_ell);
  if (kind == FKF_MATERN_32) {
    double t = 1.7320508075688772 * r * inv_ell;
    return theta * (1.0 + t) * exp(-t);
  }
  double t = 2.2360679774997896 * r * inv_ell;
  return theta * (1.0 + t + t * t * (1.0 / 3.0)) * exp(-t);
}

// Barycentric Lagrange basis at normalised coordinate x on Chebyshev nodes.
__device__ __forceinline__ void lagrange_dev(int p, const double *u, const double *w, double x,
                                             double *L) {
  double s = 0;
  int exact = -1;
  for (int a = 0; a < p; ++a) {
    double dx = x - u[a];
    if (dx == 0.0) exact = a;
    double q = w[a] / dx;
    L[a] = q;
    s += q;
  }
  if (exact >= 0) {
    for (int a = 0; a < p; ++a) L[a] = (a == exact) ? 1.0 : 0.0;
  } else {
    double is = 1.0 / s;
    for (int a = 0; a < p; ++a) L[a] *= is;
  }
}

// Offset of element (i, j) inside a lane-slice tile (in doubles).
__host__ __device__ __forceinline__ int tile_off(int i, int j) {
  int lane = (i >> 3) + 8 * (j >> 3);
  int k = 4 * (i & 7) + ((j & 7) >> 1);
  return (k * 64 + lane) * 2 + (j & 1);
}

// Gather X (caller order, ld ldx) into tree order Xt (ld n).
__global__ void k_gather(const double *__restrict__ X, int64_t ldx, int nrhs,
                         const int64_t *__restrict__ perm, int64_t n, double *__restrict__ Xt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = blockIdx.y;
  if (i < n && c < nrhs) Xt[i + n * c] = X[perm[i] + ldx * c];
}

// Near-field assembly: one wavefront per stored tile.
__global__ void __launch_bounds__(64) k_near_assemble(const double *__restrict__ pts, int64_t n,
                                                      int d, const int64_t *__restrict__ leaf_off,
                                                      const int32_t *__restrict__ bs,
                                                      const int32_t *__restrict__ bt, int kind,
                                                      double inv_ell, double theta,
                                                      double *__restrict__ blk) {
  int64_t b = blockIdx.x;
  int l = threadIdx.x;
  int ra = l & 7, cb = l >> 3;
  int s = bs[b], t = bt[b];
  int64_t s0 = leaf_off[s], ms = leaf_off[s + 1] - s0;
  int64_t t0 = leaf_off[t], mt = leaf_off[t + 1] - t0;
  double xr[8][kMaxDim], xc[8][kMaxDim];
  for (int r = 0; r < 8; ++r) {
    int64_t i = 8 * ra + r, j = 8 * cb + r;
    for (int k = 0; k < kMaxDim; ++k) {
      xr[r][k] = (i < ms && k < d) ? pts[k * n + s0 + i] : 0.0;
      xc[r][k] = (j < mt && k < d) ? pts[k * n + t0 + j] : 0.0;
    }
  }
  double2 *out = reinterpret_cast<double2 *>(blk + b * 4096);
  for (int r = 0; r < 8; ++r) {
    int i = 8 * ra + r;
    for (int cp = 0; cp < 4; ++cp) {
      double v[2];
      for (int h = 0; h < 2; ++h) {
        int c = 2 * cp + h;
        int j = 8 * cb + c;
        double r2 = 0;
        for (int k = 0; k < d; ++k) {
          double dx = xr[r][k] - xc[c][k];
          r2 += dx * dx;
        }
        v[h] = (i < ms && j < mt) ? matern_dev(sqrt(r2), kind, inv_ell, theta) : 0.0;
      }
      out[(4 * r + cp) * 64 + l] = make_double2(v[0], v[1]);
    }
  }
}

// Near field, one right-hand side, symmetric storage.  Wave w of the block
// handles tile b: row partial sums Gamma_st x_t -> part[b][0:64] and column
// partial sums Gamma_st^T x_s -> part[b][64:128].
__global__ void __launch_bounds__(256) k_near_sym1(const double *__restrict__ blk,
                                                   const int32_t *__restrict__ bs,
                                                   const int32_t *__restrict__ bt,
                                                   const int64_t *__restrict__ leaf_off,
                                                   const double *__restrict__ xt, int64_t n_blk,
                                                   double *__restrict__ part) {
  int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= n_blk) return;
  int l = threadIdx.x & 63;
  int ra = l & 7, cb = l >> 3;
  const v2d *src = reinterpret_cast<const v2d *>(blk + b * 4096);
  v2d v[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) v[k] = __builtin_nontemporal_load(src + k * 64 + l);
  int s = bs[b], t = bt[b];
  int64_t s0 = leaf_off[s], ms = leaf_off[s + 1] - s0;
  int64_t t0 = leaf_off[t], mt = leaf_off[t + 1] - t0;
  double xs[8], xc[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    int i = 8 * ra + r, j = 8 * cb + r;
    xs[r] = i < ms ? xt[s0 + i] : 0.0;
    xc[r] = j < mt ? xt[t0 + j] : 0.0;
  }
  double racc[8], cacc[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) racc[r] = cacc[r] = 0.0;
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int cp = 0; cp < 4; ++cp) {
      v2d e = v[4 * r + cp];
      racc[r] = fma(e.x, xc[2 * cp], racc[r]);
      racc[r] = fma(e.y, xc[2 * cp + 1], racc[r]);
      cacc[2 * cp] = fma(e.x, xs[r], cacc[2 * cp]);
      cacc[2 * cp + 1] = fma(e.y, xs[r], cacc[2 * cp + 1]);
    }
  // rows: reduce over lanes with equal ra (xor over cb bits 8,16,32)
#pragma unroll
  for (int m = 8; m < 64; m <<= 1)
#pragma unroll
    for (int r = 0; r < 8; ++r) racc[r] += __shfl_xor(racc[r], m);
  // columns: reduce over lanes with equal cb (xor over ra bits 1,2,4)
#pragma unroll
  for (int m = 1; m < 8; m <<= 1)
#pragma unroll
    for (int r = 0; r < 8; ++r) cacc[r] += __shfl_xor(cacc[r], m);
  double *o = part + b * 128;
  if (cb == 0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) o[8 * ra + r] = racc[r];
  }
  if (ra == 0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) o[64 + 8 * cb + r] = cacc[r];
  }
}

// Near field, several right-hand sides: one workgroup per (row leaf, 32
// columns); tiles are staged through LDS (transposed where the stored tile is
// the (t, s) half).
__global__ void __launch_bounds__(256) k_near_multi(const double *__restrict__ blk,
                                                    const int32_t *__restrict__ near_ptr,
                                                    const int32_t *__restrict__ near_idx,
                                                    const int32_t *__restrict__ bs,
                                                    const int32_t *__restrict__ bt,
                                                    const int64_t *__restrict__ leaf_off,
                                                    const double *__restrict__ xt, int64_t n,
                                                    int nrhs, double *__restrict__ yt) {
  __shared__ double A[64][65];
  __shared__ double Xs[64][33];
  int s = blockIdx.x;
  int c0 = blockIdx.y * 32;
  int tid = threadIdx.x;
  int row = tid & 63, cg = tid >> 6;
  int64_t s0 = leaf_off[s], ms = leaf_off[s + 1] - s0;
  double acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = 0.0;
  for (int e = near_ptr[s]; e < near_ptr[s + 1]; ++e) {
    int code = near_idx[e];
    int64_t b = code >> 1;
    bool trans = code & 1;
    int t = trans ? bs[b] : bt[b];
    int64_t t0 = leaf_off[t], mt = leaf_off[t + 1] - t0;
    const double2 *src = reinterpret_cast<const double2 *>(blk + b * 4096);
    for (int q = tid; q < 2048; q += 256) {
      int k = q >> 6, lane = q & 63;
      int i = 8 * (lane & 7) + (k >> 2), j = 8 * (lane >> 3) + 2 * (k & 3);
      double2 v = src[q];
      if (!trans) {
        A[i][j] = v.x;
        A[i][j + 1] = v.y;
      } else {
        A[j][i] = v.x;
        A[j + 1][i] = v.y;
      }
    }
    for (int q = tid; q < 64 * 32; q += 256) {
      int j = q & 63, c = q >> 6;
      Xs[j][c] = (j < mt && c0 + c < nrhs) ? xt[t0 + j + n * (c0 + c)] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < 64; ++j) {
      double a = A[row][j];
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] = fma(a, Xs[j][cg * 8 + c], acc[c]);
    }
    __syncthreads();
  }
  if (row < ms)
    for (int c = 0; c < 8; ++c) {
      int col = c0 + cg * 8 + c;
      if (col < nrhs) yt[s0 + row + n * col] = acc[c];
    }
}

// Far field, upward pass: xhat_c = U_c^T x_c for every far cluster c.
template <int NC>
__global__ void __launch_bounds__(256) k_far_up(const FarCluster *__restrict__ fc,
                                                const double *__restrict__ pts, int64_t n, int d,
                                                const double *__restrict__ cheb,
                                                const double *__restrict__ xt, int nrhs,
                                                double *__restrict__ xhat) {
  __shared__ double Ls[kMaxDim][64][kMaxCheb];
  __shared__ double Xs[64][NC];
  __shared__ double cu[kMaxCheb], cw[kMaxCheb];
  const FarCluster c = fc[blockIdx.x];
  const int c0 = blockIdx.y * NC;
  const int p = c.p, pd = c.pd;
  int tid = threadIdx.x;
  if (tid < p) {
    cu[tid] = cheb[p * 2 * kMaxCheb + tid];
    cw[tid] = cheb[p * 2 * kMaxCheb + kMaxCheb + tid];
  }
  const int nout = pd * NC;
  double acc[16];
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  __syncthreads();
  for (int64_t i0 = c.begin; i0 < c.end; i0 += 64) {
    int64_t cnt = min((int64_t)64, c.end - i0);
    if (tid < 64 * d) {
      int i = tid & 63, k = tid >> 6;
      if (i < cnt) {
        double x = pts[k * n + i0 + i];
        double z = c.hw[k] > 0 ? (x - c.ctr[k]) / c.hw[k] : 0.0;
        lagrange_dev(p, cu, cw, z, Ls[k][i]);
      }
    }
    for (int q = tid; q < 64 * NC; q += 256) {
      int i = q % 64, cc = q / 64;
      Xs[i][cc] = (i < cnt && c0 + cc < nrhs) ? xt[i0 + i + n * (c0 + cc)] : 0.0;
    }
    __syncthreads();
    for (int q = 0; q < 16; ++q) {
      int o = tid + 256 * q;
      if (o >= nout) break;
      int a = o % pd, cc = o / pd;
      int a0 = a % p, a1 = (a / p) % p, a2 = a / (p * p);
      double s = 0;
      for (int i = 0; i < cnt; ++i) {
        double u = Ls[0][i][a0] * Ls[1][i][a1];
        if (d == 3) u *= Ls[2][i][a2];
        s = fma(u, Xs[i][cc], s);
      }
      acc[q] += s;
    }
    __syncthreads();
  }
  for (int q = 0; q < 16; ++q) {
    int o = tid + 256 * q;
    if (o >= nout) break;
    int a = o % pd, cc = o / pd;
    if (c0 + cc < nrhs) xhat[c.coef_off * nrhs + a + (int64_t)pd * (c0 + cc)] = acc[q];
  }
}

// Far field, couplings: yhat_s = sum_{t admissible with s} K(xi_s, xi_t) xhat_t,
// with K evaluated from the node coordinates (no stored couplings).
template <int NC>
__global__ void __launch_bounds__(256) k_far_couple(const FarCluster *__restrict__ fc,
                                                    const int32_t *__restrict__ far_ptr,
                                                    const int32_t *__restrict__ far_col, int d,
                                                    const double *__restrict__ cheb, int kind,
                                                    double inv_ell, double theta,
                                                    const double *__restrict__ xhat, int nrhs,
                                                    double *__restrict__ yhat) {
  __shared__ double xi_t[kMaxCheb * kMaxCheb * kMaxCheb / 4][kMaxDim];  // up to 1024 nodes
  __shared__ double xh[4096];
  const int sidx = blockIdx.x;
  const FarCluster cs = fc[sidx];
  const int c0 = blockIdx.y * NC;
  const int tid = threadIdx.x;
  const int ps = cs.p, pds = cs.pd;
  double us[kMaxCheb];
  for (int a = 0; a < ps; ++a) us[a] = cheb[ps * 2 * kMaxCheb + a];
  for (int a0 = 0; a0 < pds; a0 += 256) {
    int a = a0 + tid;
    double xs[kMaxDim] = {0, 0, 0};
    if (a < pds) {
      int r = a;
      for (int k = 0; k < d; ++k) {
        xs[k] = cs.ctr[k] + cs.hw[k] * us[r % ps];
        r /= ps;
      }
    }
    double acc[NC];
    for (int cc = 0; cc < NC; ++cc) acc[cc] = 0.0;
    for (int e = far_ptr[sidx]; e < far_ptr[sidx + 1]; ++e) {
      const FarCluster ct = fc[far_col[e]];
      const int pt = ct.p, pdt = ct.pd;
      __syncthreads();
      for (int b = tid; b < pdt; b += 256) {
        int r = b;
        for (int k = 0; k < d; ++k) {
          xi_t[b][k] = ct.ctr[k] + ct.hw[k] * cheb[pt * 2 * kMaxCheb + (r % pt)];
          r /= pt;
        }
      }
      for (int q = tid; q < pdt * NC; q += 256) {
        int b = q % pdt, cc = q / pdt;
        xh[q] = (c0 + cc < nrhs) ? xhat[ct.coef_off * nrhs + b + (int64_t)pdt * (c0 + cc)] : 0.0;
      }
      __syncthreads();
      if (a < pds) {
        for (int b = 0; b < pdt; ++b) {
          double r2 = 0;
          for (int k = 0; k < d; ++k) {
            double dx = xs[k] - xi_t[b][k];
            r2 += dx * dx;
          }
          double kv = matern_dev(sqrt(r2), kind, inv_ell, theta);
#pragma unroll
          for (int cc = 0; cc < NC; ++cc) acc[cc] = fma(kv, xh[b + pdt * cc], acc[cc]);
        }
      }
    }
    if (a < pds)
      for (int cc = 0; cc < NC; ++cc)
        if (c0 + cc < nrhs) yhat[cs.coef_off * nrhs + a + (int64_t)pds * (c0 + cc)] = acc[cc];
  }
}

// Downward pass + near-field reduction + scatter to caller order:
// y_i = (near part) + sum over far-cluster ancestors c of leaf: U_c(x_i) yhat_c.
template <int NC>
__global__ void __launch_bounds__(256) k_finalize(
    const int64_t *__restrict__ leaf_off, const double *__restrict__ pts, int64_t n, int d,
    const double *__restrict__ cheb, const FarCluster *__restrict__ fc,
    const int32_t *__restrict__ anc_ptr, const int32_t *__restrict__ anc_idx,
    const double *__restrict__ yhat, const double *__restrict__ part,
    const int32_t *__restrict__ part_ptr, const int32_t *__restrict__ part_idx,
    const double *__restrict__ yt, const int64_t *__restrict__ perm, int nrhs,
    double *__restrict__ Y, int64_t ldy) {
  __shared__ double Ls[kMaxDim][64][kMaxCheb];
  __shared__ double yh[4096];
  __shared__ double cu[kMaxCheb], cw[kMaxCheb];
  const int leaf = blockIdx.x;
  const int c0 = blockIdx.y * NC;
  const int tid = threadIdx.x;
  const int64_t s0 = leaf_off[leaf], m = leaf_off[leaf + 1] - s0;
  const int i = tid & 63, cg = tid >> 6;
  constexpr int PER = (NC + 3) / 4;
  double acc[PER];
  for (int q = 0; q < PER; ++q) acc[q] = 0.0;
  for (int e = anc_ptr[leaf]; e < anc_ptr[leaf + 1]; ++e) {
    const FarCluster c = fc[anc_idx[e]];
    const int p = c.p, pd = c.pd;
    __syncthreads();
    if (tid < p) {
      cu[tid] = cheb[p * 2 * kMaxCheb + tid];
      cw[tid] = cheb[p * 2 * kMaxCheb + kMaxCheb + tid];
    }
    __syncthreads();
    if (tid < 64 * d) {
      int ii = tid & 63, k = tid >> 6;
      if (ii < m) {
        double x = pts[k * n + s0 + ii];
        double z = c.hw[k] > 0 ? (x - c.ctr[k]) / c.hw[k] : 0.0;
        lagrange_dev(p, cu, cw, z, Ls[k][ii]);
      }
    }
    for (int q = tid; q < pd * NC; q += 256) {
      int a = q % pd, cc = q / pd;
      yh[q] = (c0 + cc < nrhs) ? yhat[c.coef_off * nrhs + a + (int64_t)pd * (c0 + cc)] : 0.0;
    }
    __syncthreads();
    if (i < m) {
      for (int q = 0; q < PER; ++q) {
        int cc = cg + 4 * q;
        if (cc >= NC) break;
        double s = 0;
        for (int a = 0; a < pd; ++a) {
          int a0 = a % p, a1 = (a / p) % p, a2 = a / (p * p);
          double u = Ls[0][i][a0] * Ls[1][i][a1];
          if (d == 3) u *= Ls[2][i][a2];
          s = fma(u, yh[a + pd * cc], s);
        }
        acc[q] += s;
      }
    }
  }
  if (i < m) {
    for (int q = 0; q < PER; ++q) {
      int cc = cg + 4 * q;
      if (cc >= NC || c0 + cc >= nrhs) break;
      double v = acc[q];
      if (part) {
        for (int e = part_ptr[leaf]; e < part_ptr[leaf + 1]; ++e) {
          int code = part_idx[e];
          v += part[(int64_t)(code >> 1) * 128 + (code & 1) * 64 + i];
        }
      } else {
        v += yt[s0 + i + n * (c0 + cc)];
      }
      Y[perm[s0 + i] + ldy * (c0 + cc)] = v;
    }
  }
}

}  // namespace fkf

// ------------------------------------------------------------------ host ---
using namespace fkf;

extern "C" fkf_status fkf_cov_build(const double *pts_host, int64_t n, int32_t d,
                                    const fkf_kernel_params *kp, const fkf_hmat_params *hp,
                                    void *stream, fkf_cov **out) {
  return guarded([&] {
    FKF_REQUIRE(out != nullptr, "fkf_cov_build: out is NULL");
    *out = nullptr;
    FKF_REQUIRE(pts_host != nullptr && kp != nullptr && hp != nullptr,
                "fkf_cov_build: NULL argument");
    FKF_REQUIRE(n > 0, "fkf_cov_build: n must be positive");
    FKF_REQUIRE(d == 2 || d == 3, "fkf_cov_build: d must be 2 or 3");
    FKF_REQUIRE(kp->struct_size == sizeof(fkf_kernel_params), "fkf_cov_build: kernel struct_size");
    FKF_REQUIRE(hp->struct_size == sizeof(fkf_hmat_params), "fkf_cov_build: hmat struct_size");
    FKF_REQUIRE(kp->kind >= 0 && kp->kind <= 2, "fkf_cov_build: unknown kernel kind");
    FKF_REQUIRE(kp->variance > 0 && kp->length > 0, "fkf_cov_build: variance and length must be > 0");
    FKF_REQUIRE(hp->leaf_size >= 1 && hp->leaf_size <= kTile, "fkf_cov_build: leaf_size in 1..64");
    FKF_REQUIRE(hp->cheb_order >= 2 && hp->cheb_order <= kMaxCheb, "fkf_cov_build: cheb_order in 2..16");
    FKF_REQUIRE(hp->block_tol <= 0 || (hp->cheb_order_max >= hp->cheb_order &&
                                       hp->cheb_order_max <= kMaxCheb),
                "fkf_cov_build: cheb_order_max in cheb_order..16");
    FKF_REQUIRE(hp->eta > 0, "fkf_cov_build: eta must be > 0");
    FKF_REQUIRE(hp->precision == FKF_FP64, "fkf_cov_build: only FP64 precision");
    for (int64_t i = 0; i < n * d; ++i)
      FKF_REQUIRE(std::isfinite(pts_host[i]), "fkf_cov_build: non-finite coordinate");
    hipStream_t st = as_stream(stream);

    auto cov = std::make_unique<fkf_cov>();
    cov->n = n;
    cov->d = d;
    cov->kind = kp->kind;
    cov->theta = kp->variance;
    cov->ell = kp->length;
    cov->hp = *hp;
    Tree &t = cov->tree;
    t = build_tree(pts_host, n, d, hp->leaf_size);
    std::vector<std::pair<int, int>> near, far;
    partition(t, hp->eta, near, far);
    int pmax = hp->block_tol > 0 ? hp->cheb_order_max : hp->cheb_order;
    if (d == 3) pmax = std::min(pmax, 10);
    cov->level_p = choose_cheb_orders(t, pts_host, far, kp->kind, kp->length, kp->variance,
                                      std::min(hp->cheb_order, pmax), pmax, hp->block_tol);
    cov->n_leaves = (int)t.leaves.size();
    cov->n_near_pairs = (int64_t)near.size();
    cov->n_far_pairs = (int64_t)far.size();
    for (auto &pr : near) cov->covered += t.nodes[pr.first].size() * t.nodes[pr.second].size();
    for (auto &pr : far) cov->covered += t.nodes[pr.first].size() * t.nodes[pr.second].size();

    // points (tree order, SoA) and permutation
    std::vector<double> ptree((size_t)d * n);
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < d; ++k) ptree[(size_t)k * n + i] = pts_host[t.perm[i] * d + k];
    cov->pts.upload(ptree, st);
    cov->perm.upload(t.perm, st);
    std::vector<int64_t> loff(cov->n_leaves + 1);
    for (int l = 0; l < cov->n_leaves; ++l) loff[l] = t.nodes[t.leaves[l]].begin;
    loff[cov->n_leaves] = n;
    cov->leaf_off.upload(loff, st);

    // near field: symmetric half
    std::vector<int32_t> bs, bt;
    for (auto &pr : near) {
      int ls = t.nodes[pr.first].leaf, lt = t.nodes[pr.second].leaf;
      if (ls <= lt) {
        bs.push_back(ls);
        bt.push_back(lt);
      }
    }
    // order tiles by (s, t) for locality
    std::vector<size_t> ord(bs.size());
    std::iota(ord.begin(), ord.end(), (size_t)0);
    std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
      return bs[a] != bs[b] ? bs[a] < bs[b] : bt[a] < bt[b];
    });
    std::vector<int32_t> bs2(bs.size()), bt2(bs.size());
    for (size_t i = 0; i < ord.size(); ++i) {
      bs2[i] = bs[ord[i]];
      bt2[i] = bt[ord[i]];
    }
    cov->n_blk = (int64_t)bs2.size();
    std::vector<std::vector<int32_t>> plist(cov->n_leaves), nlist(cov->n_leaves);
    for (int64_t b = 0; b < cov->n_blk; ++b) {
      plist[bs2[b]].push_back((int32_t)(b * 2 + 0));
      nlist[bs2[b]].push_back((int32_t)(b * 2 + 0));
      if (bs2[b] != bt2[b]) {
        plist[bt2[b]].push_back((int32_t)(b * 2 + 1));
        nlist[bt2[b]].push_back((int32_t)(b * 2 + 1));
      }
    }
    auto to_csr = [](const std::vector<std::vector<int32_t>> &L, std::vector<int32_t> &ptr,
                     std::vector<int32_t> &idx) {
      ptr.assign(1, 0);
      idx.clear();
      for (auto &v : L) {
        idx.insert(idx.end(), v.begin(), v.end());
        ptr.push_back((int32_t)idx.size());
      }
    };
    std::vector<int32_t> pp, pi, np_, ni;
    to_csr(plist, pp, pi);
    to_csr(nlist, np_, ni);
    cov->blk_s.upload(bs2, st);
    cov->blk_t.upload(bt2, st);
    cov->part_ptr.upload(pp, st);
    cov->part_idx.upload(pi, st);
    cov->near_ptr.upload(np_, st);
    cov->near_idx.upload(ni, st);
    cov->blk.alloc((size_t)cov->n_blk * 4096);
    if (cov->n_blk > 0)
      hipLaunchKernelGGL(k_near_assemble, dim3((unsigned)cov->n_blk), dim3(64), 0, st,
                         cov->pts.p, n, d, cov->leaf_off.p, cov->blk_s.p, cov->blk_t.p,
                         cov->kind, 1.0 / cov->ell, cov->theta, cov->blk.p);
    FKF_CHECK_HIP(hipGetLastError());

    // far clusters
    std::vector<int> fidx(t.nodes.size(), -1);
    std::vector<FarCluster> fcs;
    auto far_id = [&](int node) {
      if (fidx[node] >= 0) return fidx[node];
      const Node &nd = t.nodes[node];
      FarCluster c{};
      c.begin = nd.begin;
      c.end = nd.end;
      c.p = cov->level_p[nd.level];
      c.pd = 1;
      for (int k = 0; k < d; ++k) c.pd *= c.p;
      for (int k = 0; k < kMaxDim; ++k) {
        c.ctr[k] = k < d ? 0.5 * (nd.lo[k] + nd.hi[k]) : 0.0;
        c.hw[k] = k < d ? 0.5 * (nd.hi[k] - nd.lo[k]) : 0.0;
      }
      fidx[node] = (int)fcs.size();
      fcs.push_back(c);
      return fidx[node];
    };
    std::vector<std::pair<int, int>> fpairs;
    for (auto &pr : far) fpairs.emplace_back(far_id(pr.first), far_id(pr.second));
    cov->n_fc = (int)fcs.size();
    int64_t off = 0;
    for (auto &c : fcs) {
      c.coef_off = off;
      off += c.pd;
      cov->max_pd = std::max(cov->max_pd, c.pd);
    }
    cov->n_coef = off;
    std::vector<std::vector<int32_t>> flist(cov->n_fc);
    for (auto &pr : fpairs) flist[pr.first].push_back(pr.second);
    std::vector<int32_t> fp, fcol;
    to_csr(flist, fp, fcol);
    std::vector<std::vector<int32_t>> alist(cov->n_leaves);
    for (int l = 0; l < cov->n_leaves; ++l)
      for (int nd = t.leaves[l]; nd >= 0; nd = t.nodes[nd].parent)
        if (fidx[nd] >= 0) alist[l].push_back(fidx[nd]);
    std::vector<int32_t> ap, ai;
    to_csr(alist, ap, ai);
    cov->fc.upload(fcs, st);
    cov->far_ptr.upload(fp, st);
    cov->far_col.upload(fcol, st);
    cov->anc_ptr.upload(ap, st);
    cov->anc_idx.upload(ai, st);
    std::vector<double> ch((kMaxCheb + 1) * 2 * kMaxCheb, 0.0);
    for (int p = 1; p <= kMaxCheb; ++p) cheb_nodes(p, &ch[p * 2 * kMaxCheb], &ch[p * 2 * kMaxCheb + kMaxCheb]);
    cov->cheb.upload(ch, st);
    FKF_CHECK_HIP(hipStreamSynchronize(st));
    *out = cov.release();
  });
}

extern "C" fkf_status fkf_cov_apply(fkf_cov *cov, const double *X, int64_t ldx, int32_t nrhs,
                                    double *Y, int64_t ldy, void *stream) {
  return guarded([&] {
    FKF_REQUIRE(cov != nullptr, "fkf_cov_apply: NULL handle");
    FKF_REQUIRE(nrhs >= 0, "fkf_cov_apply: nrhs < 0");
    if (nrhs == 0) return;
    FKF_REQUIRE(X != nullptr && Y != nullptr, "fkf_cov_apply: NULL array");
    FKF_REQUIRE(ldx >= cov->n && ldy >= cov->n, "fkf_cov_apply: leading dimension < n");
    hipStream_t st = as_stream(stream);
    const int64_t n = cov->n;
    cov->xt.reserve((size_t)n * nrhs);
    dim3 gg((unsigned)((n + 255) / 256), (unsigned)nrhs);
    {
      FKF_TRACE("hmat_gather", st);
      hipLaunchKernelGGL(k_gather, gg, dim3(256), 0, st, X, ldx, nrhs, cov->perm.p, n, cov->xt.p);
    }
    const bool one = (nrhs == 1);
    if (one) {
      cov->part.reserve((size_t)std::max<int64_t>(cov->n_blk, 1) * 128);
      FKF_TRACE("hmat_near_1rhs", st);
      if (cov->n_blk)
        hipLaunchKernelGGL(k_near_sym1, dim3((unsigned)((cov->n_blk + 3) / 4)), dim3(256), 0, st,
                           cov->blk.p, cov->blk_s.p, cov->blk_t.p, cov->leaf_off.p, cov->xt.p,
                           cov->n_blk, cov->part.p);
    } else {
      cov->yt.reserve((size_t)n * nrhs);
      FKF_TRACE("hmat_near_multi", st);
      hipLaunchKernelGGL(k_near_multi, dim3(cov->n_leaves, (unsigned)((nrhs + 31) / 32)), dim3(256),
                         0, st, cov->blk.p, cov->near_ptr.p, cov->near_idx.p, cov->blk_s.p,
                         cov->blk_t.p, cov->leaf_off.p, cov->xt.p, n, nrhs, cov->yt.p);
    }
    // columns per far-field workgroup: NC * max(p^d) must fit the 4096-entry LDS staging
    const int NCm = cov->max_pd <= 512 ? 8 : 4;
    if (cov->n_fc > 0) {
      cov->xhat.reserve((size_t)cov->n_coef * nrhs);
      cov->yhat.reserve((size_t)cov->n_coef * nrhs);
      FKF_TRACE(one ? "hmat_far_1rhs" : "hmat_far_multi", st);
      if (one) {
        hipLaunchKernelGGL(k_far_up<1>, dim3(cov->n_fc, 1), dim3(256), 0, st, cov->fc.p,
                           cov->pts.p, n, cov->d, cov->cheb.p, cov->xt.p, nrhs, cov->xhat.p);
        hipLaunchKernelGGL(k_far_couple<1>, dim3(cov->n_fc, 1), dim3(256), 0, st, cov->fc.p,
                           cov->far_ptr.p, cov->far_col.p, cov->d, cov->cheb.p, cov->kind,
                           1.0 / cov->ell, cov->theta, cov->xhat.p, nrhs, cov->yhat.p);
      } else {
        unsigned gy = (unsigned)((nrhs + NCm - 1) / NCm);
        if (NCm == 8) {
          hipLaunchKernelGGL(k_far_up<8>, dim3(cov->n_fc, gy), dim3(256), 0, st, cov->fc.p,
                             cov->pts.p, n, cov->d, cov->cheb.p, cov->xt.p, nrhs, cov->xhat.p);
          hipLaunchKernelGGL(k_far_couple<8>, dim3(cov->n_fc, gy), dim3(256), 0, st, cov->fc.p,
                             cov->far_ptr.p, cov->far_col.p, cov->d, cov->cheb.p, cov->kind,
                             1.0 / cov->ell, cov->theta, cov->xhat.p, nrhs, cov->yhat.p);
        } else {
          hipLaunchKernelGGL(k_far_up<4>, dim3(cov->n_fc, gy), dim3(256), 0, st, cov->fc.p,
                             cov->pts.p, n, cov->d, cov->cheb.p, cov->xt.p, nrhs, cov->xhat.p);
          hipLaunchKernelGGL(k_far_couple<4>, dim3(cov->n_fc, gy), dim3(256), 0, st, cov->fc.p,
                             cov->far_ptr.p, cov->far_col.p, cov->d, cov->cheb.p, cov->kind,
                             1.0 / cov->ell, cov->theta, cov->xhat.p, nrhs, cov->yhat.p);
        }
      }
    }
    FKF_TRACE(one ? "hmat_finalize_1rhs" : "hmat_finalize_multi", st);
    if (one) {
      hipLaunchKernelGGL(k_finalize<1>, dim3(cov->n_leaves, 1), dim3(256), 0, st,
                         cov->leaf_off.p, cov->pts.p, n, cov->d, cov->cheb.p, cov->fc.p,
                         cov->anc_ptr.p, cov->anc_idx.p, cov->yhat.p, cov->part.p,
                         cov->part_ptr.p, cov->part_idx.p, (const double *)nullptr, cov->perm.p,
                         nrhs, Y, ldy);
    } else {
      auto fin = NCm == 8 ? k_finalize<8> : k_finalize<4>;
      hipLaunchKernelGGL(fin, dim3(cov->n_leaves, (unsigned)((nrhs + NCm - 1) / NCm)),
                         dim3(256), 0, st, cov->leaf_off.p, cov->pts.p, n, cov->d, cov->cheb.p,
                         cov->fc.p, cov->anc_ptr.p, cov->anc_idx.p, cov->yhat.p,
                         (const double *)nullptr, cov->part_ptr.p, cov->part_idx.p, cov->yt.p,
                         cov->perm.p, nrhs, Y, ldy);
    }
    FKF_CHECK_HIP(hipGetLastError());
  });
}

extern "C" fkf_status fkf_cov_info(const fkf_cov *cov, fkf_cov_info_t *info) {
  return guarded([&] {
    FKF_REQUIRE(cov != nullptr && info != nullptr, "fkf_cov_info: NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->n = cov->n;
    info->dim = cov->d;
    info->n_leaves = cov->n_leaves;
    info->n_levels = cov->tree.depth + 1;
    info->n_near_blocks = cov->n_blk;
    info->n_near_pairs = cov->n_near_pairs;
    info->n_far_pairs = cov->n_far_pairs;
    info->near_bytes = cov->n_blk * 4096 * (int64_t)sizeof(double);
    info->far_coef_per_rhs = cov->n_coef;
    for (int l = 0; l < 32 && l < (int)cov->level_p.size(); ++l) info->cheb_p[l] = cov->level_p[l];
    info->covered_entries = cov->covered;
  });
}

extern "C" fkf_status fkf_cov_perm(const fkf_cov *cov, int64_t *perm_host) {
  return guarded([&] {
    FKF_REQUIRE(cov != nullptr && perm_host != nullptr, "fkf_cov_perm: NULL argument");
    std::copy(cov->tree.perm.begin(), cov->tree.perm.end(), perm_host);
  });
}

extern "C" void fkf_cov_destroy(fkf_cov *cov) {
  if (!cov) return;
  (void)hipDeviceSynchronize();
  delete cov;
}

extern "C" fkf_status fkf_cov_plan(const double *pts_host, int64_t n, int32_t d,
                                   const fkf_kernel_params *kp, const fkf_hmat_params *hp,
                                   fkf_cov_info_t *info) {
  return guarded([&] {
    FKF_REQUIRE(pts_host && kp && hp && info, "fkf_cov_plan: NULL argument");
    FKF_REQUIRE(n > 0 && (d == 2 || d == 3), "fkf_cov_plan: bad n or d");
    FKF_REQUIRE(hp->leaf_size >= 1 && hp->leaf_size <= kTile, "fkf_cov_plan: leaf_size in 1..64");
    FKF_REQUIRE(hp->cheb_order >= 2 && hp->cheb_order <= kMaxCheb, "fkf_cov_plan: cheb_order");
    FKF_REQUIRE(hp->eta > 0, "fkf_cov_plan: eta must be > 0");
    Tree t = build_tree(pts_host, n, d, hp->leaf_size);
    std::vector<std::pair<int, int>> near, far;
    partition(t, hp->eta, near, far);
    int pmax = hp->block_tol > 0 ? hp->cheb_order_max : hp->cheb_order;
    if (d == 3) pmax = std::min(pmax, 10);
    auto lp = choose_cheb_orders(t, pts_host, far, kp->kind, kp->length, kp->variance,
                                 std::min(hp->cheb_order, pmax), pmax, hp->block_tol);
    std::memset(info, 0, sizeof(*info));
    info->n = n;
    info->dim = d;
    info->n_leaves = (int)t.leaves.size();
    info->n_levels = t.depth + 1;
    int64_t nb = 0, cov = 0;
    for (auto &pr : near) {
      if (t.nodes[pr.first].leaf <= t.nodes[pr.second].leaf) ++nb;
      cov += t.nodes[pr.first].size() * t.nodes[pr.second].size();
    }
    for (auto &pr : far) cov += t.nodes[pr.first].size() * t.nodes[pr.second].size();
    info->n_near_blocks = nb;
    info->n_near_pairs = (int64_t)near.size();
    info->n_far_pairs = (int64_t)far.size();
    info->near_bytes = nb * 4096 * (int64_t)sizeof(double);
    info->covered_entries = cov;
    for (int l = 0; l < 32 && l < (int)lp.size(); ++l) info->cheb_p[l] = lp[l];
  });
}

namespace fkf {
double cov_variance(const fkf_cov *cov) { return cov->theta; }
int64_t cov_n(const fkf_cov *cov) { return cov->n; }
}  // namespace fkf
