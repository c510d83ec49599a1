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
#include <map>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace fkf {

struct FarCluster {
  int64_t begin, end;
  int64_t coef_off;   // offset (in units of coefficients) of this cluster
  int64_t lag_off;    // offset of its points' Lagrange values in the table
  int32_t p, pd;      // nodes per dimension, p^d
  double ctr[kMaxDim], hw[kMaxDim];
};

// Upward work item: a chunk of <= kUpChunk points of one far cluster.
constexpr int64_t kUpChunk = 256;
constexpr int64_t kUpChunkM = 1024;   // chunk for the several-column path
struct UpItem {
  int32_t fc;       // far cluster
  int32_t pad;
  int64_t begin, end;
  int64_t poff;     // offset of this item's partial in the upward partial buffer
};

// Unordered admissible pair {s, t} (s < t) with the offset of its partials,
// ncb = ceil(pd_t / 64) vectors of length pd_s for s followed by
// nrb = ceil(pd_s / 32) vectors of length pd_t for t, and the offset koff of
// its stored coupling matrix K(xi_s, xi_t) (pd_s x pd_t, row-major) when
// couplings are stored.
struct PairItem {
  int32_t s, t;
  int64_t off;
  int64_t koff;
};

// Rows of K per coupling sub-block (columns: 64, one per lane).
constexpr int kRowBlk = 32;

// One kRowBlk x 64 (at most) sub-block (rb, cb) of the couplings of a pair.
struct CoupleItem {
  int32_t pair;
  int16_t rb, cb;
};

// One-column couplings grouped by coupling sequence: far clusters whose far
// lists, sorted by stored matrix, use the same sequence of matrices (the
// interior clusters of a level of a regular grid) form a group, and one work
// item multiplies a 64-row block of every matrix of the sequence with the
// moments of the matching partners of up to kGrpSlots targets of the group.
struct GroupItem {
  int32_t seq;     // first entry of the group's sequence in grp_koff / grp_pdt
  int32_t len;     // matrices in the sequence
  int32_t pd;      // coefficients of each target (columns of every stored matrix)
  int32_t rb;      // 64-row block of the targets' coefficients
  int32_t slot0;   // first target slot of the item (grp_tcoef)
  int32_t nslot;   // targets of the item (<= kGrpSlots)
  int32_t xbase;   // grp_xoff row of slot0 (rows of len entries per slot)
  int32_t pad;
};
constexpr int kGrpSlots = 8;

// A 64-row block rb of the coefficients of far cluster s (several-column
// couplings), or of upward item u (several-column upward pass).
struct CoupleMItem {
  int32_t s, rb;
};

// Couplings are stored (evaluated once at build) when they take at most this
// many bytes; otherwise every product evaluates them again.
constexpr int64_t kMaxCouplingBytes = int64_t(8) << 30;

// Device workspaces of one product block (carved from one allocation).
struct ApplyWs {
  double *xt = nullptr;         // gathered columns, tree order
  double *part = nullptr;       // one column: near-field partials, 128 per stored block
  double *xhat = nullptr;       // far-cluster moments U_c^T x_c
  double *yhat = nullptr;       // far-cluster coupled coefficients
  double *part_up = nullptr;    // one column: upward chunk partials
  double *part_pair = nullptr;  // one column: coupling partials (couplings evaluated)
  double *part_up_m = nullptr;  // several columns: upward chunk partials
};

}  // namespace fkf

struct fkf_cov {
  int64_t n = 0;
  int d = 2;
  int kind = 0;
  double theta = 1, ell = 1;
  double amp = 1;   // multiplier of the kernel shape: theta, or theta / ell for a length derivative
  fkf_hmat_params hp{};
  fkf::Tree tree;
  std::vector<int> level_p;
  int n_leaves = 0;
  int64_t n_blk = 0, n_near_pairs = 0, n_far_pairs = 0, n_coef = 0, covered = 0;
  int64_t n_interp = 0;   // sum over far clusters of |c| * p^d
  int n_fc = 0;
  int max_pd = 1;
  fkf::DevBuf<int64_t> perm;
  fkf::DevBuf<double> pts;          // d x n, tree order
  fkf::DevBuf<int64_t> leaf_off;    // n_leaves + 1
  fkf::DevBuf<int32_t> blk_s, blk_t;
  fkf::DevBuf<double> blk;          // n_blk x 4096 (FP64 mode)
  fkf::DevBuf<float> blk32;         // n_blk x 4096 (mixed mode)
  bool mixed = false;
  fkf::DevBuf<int32_t> part_ptr, part_idx;   // per leaf: entries blk*2 + side
  fkf::DevBuf<int32_t> near_ptr, near_idx;   // per leaf: entries blk*2 + transposed
  fkf::DevBuf<int32_t> near_src;             // source leaf of each near_idx entry
  // tiles of the ordered near pairs (near_idx order) in FP64 MFMA A-operand
  // order, for the several-column product (FP32 in the mixed mode)
  fkf::DevBuf<double> frag;
  fkf::DevBuf<float> frag32;
  fkf::DevBuf<fkf::FarCluster> fc;
  fkf::DevBuf<int32_t> far_ptr, far_col;     // partners per target far cluster
  fkf::DevBuf<fkf::CoupleMItem> cm_items;     // several-column coupling blocks, costliest first
  int64_t n_cm_items = 0;
  bool cm_all = true;                         // every far cluster has a partner
  fkf::DevBuf<int32_t> anc_ptr, anc_idx;     // far-cluster ancestors of each leaf
  fkf::DevBuf<double> cheb;                  // [p][a] nodes and weights
  // one-column far field work lists
  fkf::DevBuf<fkf::UpItem> up_items;
  fkf::DevBuf<int32_t> up_ptr;               // items of each far cluster
  fkf::DevBuf<fkf::PairItem> pairs;          // unordered admissible pairs (large first)
  fkf::DevBuf<fkf::PairItem> upairs;         // one pair per distinct stored coupling matrix
  int64_t n_upairs = 0;
  int64_t n_kst = 0;                         // entries of the distinct stored coupling matrices
  int64_t n_kpair = 0;                       // entries of the coupling matrices of all pairs
  fkf::DevBuf<double> kst;                   // stored couplings (FP64 mode)
  fkf::DevBuf<float> kst32;                  // stored couplings (mixed mode)
  bool stored = false;
  fkf::DevBuf<fkf::CoupleItem> citems;       // 64 x 64 coupling sub-blocks
  fkf::DevBuf<int64_t> far_koff;             // stored matrix of each far list entry
  // grouped one-column couplings (stored couplings shared by many targets)
  fkf::DevBuf<fkf::GroupItem> grp_items;
  fkf::DevBuf<int64_t> grp_koff;             // sequences of stored matrices
  fkf::DevBuf<int32_t> grp_pdt;              // partner coefficients of each sequence entry
  fkf::DevBuf<int32_t> grp_tcoef;            // coef_off of the target of each slot
  fkf::DevBuf<int32_t> grp_xoff;             // coef_off of the partner, per slot and entry
  int64_t n_grp_items = 0, n_grp_groups = 0;
  bool grouped = false;
  int64_t n_citems = 0;
  fkf::DevBuf<int32_t> cp_ptr;               // pair partials of each far cluster
  fkf::DevBuf<int64_t> cp_off;
  int64_t n_up_items = 0, n_part_up = 0, n_pairs = 0, n_part_pair = 0;
  fkf::DevBuf<double> lag;                   // Lagrange values: per far cluster, point, axis,
                                             // PMax nodes (several-column upward pass)
  fkf::DevBuf<fkf::UpItem> up_items_m;       // several-column upward chunks
  fkf::DevBuf<fkf::CoupleMItem> up_blocks_m; // (chunk, 64-row block), costliest first
  int64_t n_up_blocks_m = 0;
  fkf::DevBuf<int32_t> up_ptr_m;
  int64_t n_up_items_m = 0, n_part_up_m = 0;
  // sparse right-hand sides (rows of a sparse matrix as the columns): tree
  // position of every point and the leaf range [first, end) of every far
  // cluster; sp_ok when every far cluster is a whole range of leaves
  fkf::DevBuf<int32_t> iperm, fc_leaf;
  bool sp_ok = false;
  // workspace
  fkf::DevBuf<double> ws;                // product workspace (grown on demand)
  fkf::DevBuf<int32_t> sp_tix, sp_cnt;   // sparse rows in tree order, per-leaf counts
  fkf::DevBuf<int32_t> sp_nzb;           // nonzero 16-column blocks of the moments
  fkf::DevBuf<int32_t> sp_ynz;           // nonzero 16-column blocks of Yhat
  fkf::DevBuf<int32_t> sp_plist, sp_pcnt; // partners with nonzero moments per 256 columns
  fkf::DevBuf<double> sp_val;
  // fork/join of the near field onto a second stream
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  ~fkf_cov() {
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
  }
};

namespace fkf {

// ------------------------------------------------------------ device code ---
// Scale c of the scaled distance t = c r / ell (c = 1, sqrt 3, sqrt 5 for
// nu = 1/2, 3/2, 5/2; the length derivatives share their kernel's scale).
__host__ __device__ __forceinline__ double kernel_c(int kind) {
  const int b = kind % 3;
  return b == 0 ? 1.0 : (b == 1 ? 1.7320508075688772 : 2.2360679774997896);
}

// Shape of the kernel as a function of t (eq. maternfamily, half-integer
// closed forms) and, for the length-derivative kinds, -t C'(t): the factor
// that, times variance / ell, gives d/d ell of variance C(c r / ell).
template <typename T>
__device__ __forceinline__ T kernel_shape(int kind, T t, T ex) {
  switch (kind) {
    case FKF_MATERN_12: return ex;
    case FKF_MATERN_32: return t * ex + ex;
    case FKF_MATERN_52: return (t * (T)(1.0 / 3.0) + (T)1) * t * ex + ex;
    case FKF_MATERN_12_DLENGTH: return t * ex;
    case FKF_MATERN_32_DLENGTH: return t * t * ex;
    default: return t * t * ((T)1 + t) * ex * (T)(1.0 / 3.0);
  }
}

// amp * shape at distance r (near-field assembly; amp is the variance, or
// variance / ell for a length derivative).
__device__ __forceinline__ double matern_dev(double r, int kind, double inv_ell, double amp) {
  const double t = kernel_c(kind) * r * inv_ell;
  return amp * kernel_shape<double>(kind, t, exp(-t));
}

// Kernel entry amp * shape(t) from the square t2 of the scaled distance.
// F32: evaluated with the FP32 hardware square root and exponential (mixed
// precision).
template <bool F32>
__device__ __forceinline__ double kernel_t2(double t2, int kind, double amp) {
  if (F32) {
    const float t = __fsqrt_rn((float)t2);
    return amp * (double)kernel_shape<float>(kind, t, __expf(-t));
  } else {
    const double t = sqrt_pos(t2);
    return amp * kernel_shape<double>(kind, t, exp_nonpos(-t));
  }
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

// FP32 near-field tile: slice k (16 slices of 1 KiB) holds four consecutive
// entries (row 8ra + k/2, columns 8cb + 4(k%2) .. +3) of each lane's sub-tile.
__global__ void __launch_bounds__(64) k_near_assemble32(const double *__restrict__ pts, int64_t n,
                                                        int d, const int64_t *__restrict__ leaf_off,
                                                        const int32_t *__restrict__ bs,
                                                        const int32_t *__restrict__ bt, int kind,
                                                        double inv_ell, double theta,
                                                        float *__restrict__ blk) {
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
  float4 *out = reinterpret_cast<float4 *>(blk + b * 4096);
  for (int r = 0; r < 8; ++r) {
    int i = 8 * ra + r;
    for (int cq = 0; cq < 2; ++cq) {
      float v[4];
      for (int h = 0; h < 4; ++h) {
        int c = 4 * cq + h;
        int j = 8 * cb + c;
        double r2 = 0;
        for (int k = 0; k < d; ++k) {
          double dx = xr[r][k] - xc[c][k];
          r2 += dx * dx;
        }
        v[h] = (i < ms && j < mt) ? (float)matern_dev(sqrt(r2), kind, inv_ell, theta) : 0.0f;
      }
      out[(2 * r + cq) * 64 + l] = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
}

// One right-hand side, FP32 tiles (products and sums in FP64); otherwise as
// k_near_sym1 below.
__global__ void __launch_bounds__(256) k_near_sym1_32(const float *__restrict__ blk,
                                                      const int32_t *__restrict__ bs,
                                                      const int32_t *__restrict__ bt,
                                                      const int64_t *__restrict__ leaf_off,
                                                      const double *__restrict__ xt, int64_t n_blk,
                                                      double *__restrict__ part) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= n_blk) return;
  int l = threadIdx.x & 63;
  int ra = l & 7, cb = l >> 3;
  const v4f *src = reinterpret_cast<const v4f *>(blk + b * 4096);
  v4f v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = __builtin_nontemporal_load(src + k * 64 + l);
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
    for (int cq = 0; cq < 2; ++cq) {
      v4f e = v[2 * r + cq];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const double ev = (double)e[h];
        racc[r] = fma(ev, xc[4 * cq + h], racc[r]);
        cacc[4 * cq + h] = fma(ev, xs[r], cacc[4 * cq + h]);
      }
    }
#pragma unroll
  for (int m = 8; m < 64; m <<= 1)
#pragma unroll
    for (int r = 0; r < 8; ++r) racc[r] += __shfl_xor(racc[r], m);
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

// ------------------------------------------------ one-column far field ---
// Lagrange basis with compile-time bound PM (loops fully unrolled so that L
// stays in registers); u, w point to the node/weight table of p nodes.
template <int PM>
__device__ __forceinline__ void lagrange_reg(int p, const double *__restrict__ u,
                                             const double *__restrict__ w, double x,
                                             double (&L)[PM]) {
  double s = 0;
  int exact = -1;
#pragma unroll
  for (int a = 0; a < PM; ++a) {
    L[a] = 0.0;
    if (a < p) {
      double dx = x - u[a];
      if (dx == 0.0) exact = a;
      double q = w[a] / dx;
      L[a] = q;
      s += q;
    }
  }
  if (exact >= 0) {
#pragma unroll
    for (int a = 0; a < PM; ++a) L[a] = (a == exact) ? 1.0 : 0.0;
  } else {
    double is = 1.0 / s;
#pragma unroll
    for (int a = 0; a < PM; ++a) L[a] *= is;
  }
}

// Lagrange values at the p <= PM Chebyshev nodes u (first kind) in product
// form, without divisions: L_a(x) = w'_a prod_{b != a} (x - u_b) with
// w'_a = 1 / prod_{b != a} (u_a - u_b) = (2^(p-1) / p) (-1)^a sin(theta_a),
// i.e. the stored normalised weights w_a times 2^(p-1) / p, and the products
// taken as prefix times suffix (3p multiplications; each L_a to ~2p rounding
// errors; at a node x = u_a the others vanish exactly).  L[a] = 0 for
// a >= p.  For x in [-1, 1].
template <int PM>
__device__ __forceinline__ void lagrange_prod(int p, const double *__restrict__ u,
                                              const double *__restrict__ w, double x,
                                              double (&L)[PM]) {
  double d[PM], pre[PM];
  double acc = 1.0;
#pragma unroll
  for (int a = 0; a < PM; ++a) {
    d[a] = a < p ? x - u[a] : 1.0;
    pre[a] = acc;                 // prod_{b < a} (x - u_b)
    acc *= d[a];
  }
  const double sc = __builtin_ldexp(1.0, p - 1) / p;
  double suf = 1.0;               // prod_{b > a} (x - u_b)
#pragma unroll
  for (int a = PM - 1; a >= 0; --a) {
    L[a] = a < p ? sc * w[a] * pre[a] * suf : 0.0;
    suf *= d[a];
  }
}

// Barycentric Lagrange values at p <= PM Chebyshev nodes (L[a] = 0 for
// a >= p) with Newton-refined hardware reciprocals in place of divisions.
template <int PM>
__device__ __forceinline__ void lagrange_any(int p, const double *__restrict__ u,
                                             const double *__restrict__ w, double x,
                                             double (&L)[PM]) {
  double s = 0;
  int exact = -1;
#pragma unroll
  for (int a = 0; a < PM; ++a) {
    L[a] = 0.0;
    if (a < p) {
      const double dx = x - u[a];
      if (dx == 0.0) exact = a;
      const double q = w[a] * rcp_nr(dx == 0.0 ? 1.0 : dx);
      L[a] = q;
      s += q;
    }
  }
  if (exact >= 0) {
#pragma unroll
    for (int a = 0; a < PM; ++a) L[a] = (a == exact) ? 1.0 : 0.0;
  } else {
    const double is = rcp_nr(s);
#pragma unroll
    for (int a = 0; a < PM; ++a) L[a] *= is;
  }
}

template <int D> struct PMax { static constexpr int v = D == 2 ? kMaxCheb : 10; };

// Upward: one wavefront per chunk of <= kUpChunk points of a far cluster; the
// chunk's partial U_c^T x_c goes to part_up, reduced per cluster afterwards.

template <int D>
__global__ void __launch_bounds__(64) k_up1(const UpItem *__restrict__ items,
                                            const FarCluster *__restrict__ fc,
                                            const double *__restrict__ pts, int64_t n,
                                            const double *__restrict__ cheb,
                                            const double *__restrict__ xt,
                                            double *__restrict__ part_up) {
  constexpr int PM = PMax<D>::v;
  constexpr int QMAX = (D == 2 ? 256 : 1000 + 63) / 64;
  __shared__ double Ls[D][64][PM + 1];
  __shared__ double Xs[64];
  const UpItem it = items[blockIdx.x];
  const FarCluster c = fc[it.fc];
  const int p = c.p, pd = c.pd;
  const int l = threadIdx.x;
  const double *cu = cheb + p * 2 * kMaxCheb;
  int oa[QMAX][D];
  double acc[QMAX];
  const int nq = (pd + 63) / 64;
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    acc[q] = 0.0;
    int o = l + 64 * q, r = o < pd ? o : 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      oa[q][k] = r % p;
      r /= p;
    }
  }
  for (int64_t i0 = it.begin; i0 < it.end; i0 += 64) {
    const int cnt = (int)min((int64_t)64, it.end - i0);
    if (l < cnt) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        double x = pts[k * n + i0 + l];
        double z = c.hw[k] > 0 ? (x - c.ctr[k]) / c.hw[k] : 0.0;
        double L[PM];
        lagrange_reg<PM>(p, cu, cu + kMaxCheb, z, L);
#pragma unroll
        for (int a = 0; a < PM; ++a) Ls[k][l][a] = L[a];
      }
      Xs[l] = xt[i0 + l];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      if (q < nq) {
        double s = 0;
        if (D == 2) {
          const int a0 = oa[q][0], a1 = oa[q][1];
          for (int i = 0; i < cnt; ++i) s = fma(Ls[0][i][a0] * Ls[1][i][a1], Xs[i], s);
        } else {
          const int a0 = oa[q][0], a1 = oa[q][1], a2 = oa[q][D - 1];
          for (int i = 0; i < cnt; ++i)
            s = fma(Ls[0][i][a0] * Ls[1][i][a1] * Ls[D - 1][i][a2], Xs[i], s);
        }
        acc[q] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    int o = l + 64 * q;
    if (q < nq && o < pd) part_up[it.poff + o] = acc[q];
  }
}

// Sum the chunk partials of each far cluster (fixed order).
__global__ void __launch_bounds__(256) k_up_reduce(const FarCluster *__restrict__ fc, int n_fc,
                                                   const int32_t *__restrict__ item_ptr,
                                                   const UpItem *__restrict__ items,
                                                   const double *__restrict__ part_up,
                                                   double *__restrict__ xhat) {
  // one wavefront per far cluster; the cluster's chunk partials are
  // consecutive (stride pd), summed in chunk order with the loads of sixteen
  // chunks in flight
  const int c = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (c >= n_fc) return;
  const int l = threadIdx.x & 63;
  const FarCluster f = fc[c];
  const int i0 = item_ptr[c], cnt = item_ptr[c + 1] - i0;
  const int pd = f.pd;
  const double *src = part_up + items[i0].poff;
  for (int a = l; a < pd; a += 64) {
    double s = 0;
    int k = 0;
    for (; k + 16 <= cnt; k += 16) {
      double t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) t[u] = src[(int64_t)(k + u) * pd + a];
#pragma unroll
      for (int u = 0; u < 16; ++u) s += t[u];
    }
    for (; k < cnt; ++k) s += src[(int64_t)k * pd + a];
    xhat[f.coef_off + a] = s;
  }
}

// Row sums of a 32 x 64 block held as v[a] = term of row a on every lane:
// afterwards lane l (and l ^ 32) holds the sum over all 64 lanes of row
// l & 31 in v[0] (a fold of the two half-waves, then a butterfly
// reduce-scatter, 63 shuffles in all).  A macro, so that v stays in registers.
#define FKF_ROW_SUMS_32(v, l)                                         \
  do {                                                                \
    _Pragma("unroll") for (int i_ = 0; i_ < 32; ++i_) v[i_] += __shfl_xor(v[i_], 32); \
    _Pragma("unroll") for (int m_ = 16; m_ >= 1; m_ >>= 1) {          \
      const bool up_ = ((l) & m_) != 0;                               \
      _Pragma("unroll") for (int i_ = 0; i_ < m_; ++i_) {             \
        const double keep_ = up_ ? v[i_ + m_] : v[i_];                \
        const double send_ = up_ ? v[i_] : v[i_ + m_];                \
        v[i_] = keep_ + __shfl_xor(send_, m_);                        \
      }                                                               \
    }                                                                 \
  } while (0)

// Couplings over unordered admissible pairs {s, t}, evaluated in every
// product, in sub-blocks of at most 32 x 64 entries of K(xi_s, xi_t) (rows:
// nodes of s, columns: nodes of t), one wavefront per sub-block and four per
// workgroup.  Lane b owns column b of the sub-block: it evaluates K[a][b] for
// every row a, accumulates (K^T xhat_s)[b] in a register and keeps the 32 row
// terms K[a][b] xhat_t[b], reduced across the wavefront by row_sums_32.
// Sub-block (rb, cb) writes its row sums into the cb-th partial vector of s
// and its column sums into the rb-th partial vector of t (every entry of
// every partial is written by exactly one sub-block).
template <int D, bool F32>
__global__ void __launch_bounds__(256) k_couple_blk(const CoupleItem *__restrict__ items,
                                                    int64_t n_items,
                                                    const PairItem *__restrict__ pairs,
                                                    const FarCluster *__restrict__ fc,
                                                    const double *__restrict__ cheb, int kind,
                                                    double inv_ell, double theta,
                                                    const double *__restrict__ xhat,
                                                    double *__restrict__ part_pair) {
  __shared__ double xi[4][D][64];
  __shared__ double xsv[4][64];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + w;
  if (q >= n_items) return;   // whole wavefront leaves together
  const CoupleItem it = items[q];
  const PairItem pr = pairs[it.pair];
  const FarCluster cs = fc[pr.s], ct = fc[pr.t];
  const int ps = cs.p, pt = ct.p, pds = cs.pd, pdt = ct.pd;
  const int r0 = kRowBlk * it.rb, c0 = 64 * it.cb;
  const int rows = min(kRowBlk, pds - r0), cols = min(64, pdt - c0);
  const int ncb = (pdt + 63) >> 6;
  const double sq = kernel_c(kind);
  const double scale = sq * inv_ell;
  const double *us = cheb + ps * 2 * kMaxCheb, *ut = cheb + pt * 2 * kMaxCheb;
  if (l < rows) {
    int r = r0 + l;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      xi[w][k][l] = scale * (cs.ctr[k] + cs.hw[k] * us[r % ps]);
      r /= ps;
    }
    xsv[w][l] = xhat[cs.coef_off + r0 + l];
  }
  const bool col_ok = l < cols;
  double xb[D];
  {
    int r = col_ok ? c0 + l : 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      xb[k] = scale * (ct.ctr[k] + ct.hw[k] * ut[r % pt]);
      r /= pt;
    }
  }
  const double xtb = col_ok ? xhat[ct.coef_off + c0 + l] : 0.0;
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  double v[kRowBlk];
  double cacc = 0.0;
#pragma unroll
  for (int a = 0; a < kRowBlk; ++a) {
    v[a] = 0.0;
    if (a < rows) {
      double dx = xi[w][0][a] - xb[0];
      double t2 = dx * dx;
#pragma unroll
      for (int k = 1; k < D; ++k) {
        dx = xi[w][k][a] - xb[k];
        t2 = fma(dx, dx, t2);
      }
      const double kv = col_ok ? kernel_t2<F32>(t2, kind, theta) : 0.0;
      v[a] = kv * xtb;
      cacc = fma(kv, xsv[w][a], cacc);
    }
  }
  FKF_ROW_SUMS_32(v, l);
  if (l < rows) part_pair[pr.off + (int64_t)it.cb * pds + r0 + l] = v[0];
  if (col_ok) part_pair[pr.off + (int64_t)ncb * pds + (int64_t)it.rb * pdt + c0 + l] = cacc;
}

// One column with stored couplings, target-major: yhat[c.coef_off + a] = sum
// over the partners t of far cluster c of sum_b K(xi_t, xi_c)[b][a]
// xhat[t.coef_off + b], the matrix stored (for the geometry of the ordered
// pair) row-major with the partner's nodes as rows, so that lanes over a read
// it coalesced.  One workgroup per (far cluster, block of 64 coefficients):
// wavefront w takes the partners e = w, w + 4, ... of the far list (eight
// rows of K in flight), and the four partial sums are added in wavefront
// order through LDS (fixed order, deterministic).
template <typename KT>
__global__ void __launch_bounds__(256) k_couple_rows1(const FarCluster *__restrict__ fc,
                                                      const int32_t *__restrict__ far_ptr,
                                                      const int32_t *__restrict__ far_col,
                                                      const int64_t *__restrict__ far_koff,
                                                      const KT *__restrict__ kst,
                                                      const double *__restrict__ xhat,
                                                      double *__restrict__ yhat) {
  __shared__ double ps[4][64];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
  const int c = blockIdx.x;
  const FarCluster cs = fc[c];
  const int a = 64 * blockIdx.y + l;
  if (64 * (int)blockIdx.y >= cs.pd) return;   // whole workgroup leaves together
  const int ar = a < cs.pd ? a : 0;
  double acc = 0.0;
  for (int e = far_ptr[c] + w; e < far_ptr[c + 1]; e += 4) {
    const FarCluster ct = fc[far_col[e]];
    const KT *K = kst + far_koff[e] + ar;
    const double *x = xhat + ct.coef_off;
    int b = 0;
    for (; b + 8 <= ct.pd; b += 8) {
      double k[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) k[u] = (double)K[(int64_t)(b + u) * cs.pd];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = fma(k[u], x[b + u], acc);
    }
    for (; b < ct.pd; ++b) acc = fma((double)K[(int64_t)b * cs.pd], x[b], acc);
  }
  ps[w][l] = acc;
  __syncthreads();
  if (w == 0 && a < cs.pd) yhat[cs.coef_off + a] = ((ps[0][l] + ps[1][l]) + ps[2][l]) + ps[3][l];
}

// Build-time evaluation of the coupling matrices K(xi_s, xi_t) of every
// unordered admissible pair (one workgroup per pair), with the same entry
// formula as the product kernels.
template <int D, bool F32>
__global__ void __launch_bounds__(256) k_couple_store(const PairItem *__restrict__ pairs,
                                                      const FarCluster *__restrict__ fc,
                                                      const double *__restrict__ cheb, int kind,
                                                      double inv_ell, double theta,
                                                      void *__restrict__ kst) {
  typedef typename std::conditional<F32, float, double>::type KT;
  const PairItem pr = pairs[blockIdx.x];
  const FarCluster cs = fc[pr.s], ct = fc[pr.t];
  const int ps = cs.p, pt = ct.p, pds = cs.pd, pdt = ct.pd;
  const double sq = kernel_c(kind);
  const double scale = sq * inv_ell;
  const double *us = cheb + ps * 2 * kMaxCheb, *ut = cheb + pt * 2 * kMaxCheb;
  KT *dst = reinterpret_cast<KT *>(kst) + pr.koff;
  for (int64_t e = threadIdx.x; e < (int64_t)pds * pdt; e += 256) {
    int ra = (int)(e / pdt), rb = (int)(e % pdt);
    double t2 = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double xa = scale * (cs.ctr[k] + cs.hw[k] * us[ra % ps]);
      const double xb = scale * (ct.ctr[k] + ct.hw[k] * ut[rb % pt]);
      ra /= ps;
      rb /= pt;
      const double dx = xa - xb;
      t2 = k == 0 ? dx * dx : fma(dx, dx, t2);
    }
    dst[e] = (KT)kernel_t2<F32>(t2, kind, theta);
  }
}

// yhat_c = sum of the pair partials that belong to far cluster c (fixed order).
__global__ void __launch_bounds__(256) k_couple_reduce(const FarCluster *__restrict__ fc,
                                                       int n_fc,
                                                       const int32_t *__restrict__ cp_ptr,
                                                       const int64_t *__restrict__ cp_off,
                                                       const double *__restrict__ part_pair,
                                                       double *__restrict__ yhat) {
  // one wavefront per far cluster, partials summed in list order with eight
  // loads in flight
  const int c = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (c >= n_fc) return;
  const int l = threadIdx.x & 63;
  const FarCluster f = fc[c];
  const int e0 = cp_ptr[c], e1 = cp_ptr[c + 1];
  for (int a = l; a < f.pd; a += 64) {
    double s = 0;
    int e = e0;
    for (; e + 8 <= e1; e += 8) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = part_pair[cp_off[e + u] + a];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += t[u];
    }
    for (; e < e1; ++e) s += part_pair[cp_off[e] + a];
    yhat[f.coef_off + a] = s;
  }
}

// Sum, in list order, of the near-field partials of point i of a leaf
// (entries e0..e1 of part_idx: block * 2 + side); the loads of eight entries
// are issued together.
__device__ __forceinline__ double near_partials(const double *__restrict__ part, int e0, int e1,
                                                const int32_t *__restrict__ part_idx, int i) {
  double v = 0;
  int e = e0;
  for (; e + 8 <= e1; e += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int code = part_idx[e + u];
      t[u] = part[(int64_t)(code >> 1) * 128 + (code & 1) * 64 + i];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) v += t[u];
  }
  for (; e < e1; ++e) {
    const int code = part_idx[e];
    v += part[(int64_t)(code >> 1) * 128 + (code & 1) * 64 + i];
  }
  return v;
}

// Downward pass + near-field partials + scatter, one column.  Four waves split
// the far ancestors of the leaf; lane i owns point i; the tensor Lagrange
// contraction is factorised per axis.
template <int D>
__global__ void __launch_bounds__(256) k_final1(
    const int64_t *__restrict__ leaf_off, const double *__restrict__ pts, int64_t n,
    const double *__restrict__ cheb, const FarCluster *__restrict__ fc,
    const int32_t *__restrict__ anc_ptr, const int32_t *__restrict__ anc_idx,
    const double *__restrict__ yhat, const double *__restrict__ part,
    const int32_t *__restrict__ part_ptr, const int32_t *__restrict__ part_idx,
    const int64_t *__restrict__ perm, double *__restrict__ Y) {
  constexpr int PM = PMax<D>::v;
  __shared__ double wsum[4][64];
  const int leaf = blockIdx.x;
  const int tid = threadIdx.x, w = tid >> 6, i = tid & 63;
  const int64_t s0 = leaf_off[leaf], m = leaf_off[leaf + 1] - s0;
  double acc = 0;
  if (i < m) {
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = pts[k * n + s0 + i];
    for (int e = anc_ptr[leaf] + w; e < anc_ptr[leaf + 1]; e += 4) {
      const FarCluster c = fc[__builtin_amdgcn_readfirstlane(anc_idx[e])];
      const int p = c.p;
      const double *cu = cheb + p * 2 * kMaxCheb;
      const double *yh = yhat + c.coef_off;
      double L[D][PM];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        double z = c.hw[k] > 0 ? (x[k] - c.ctr[k]) / c.hw[k] : 0.0;
        lagrange_reg<PM>(p, cu, cu + kMaxCheb, z, L[k]);
      }
      double s = 0;
      if (D == 2) {
#pragma unroll
        for (int a1 = 0; a1 < PM; ++a1) {
          if (a1 < p) {
            double t = 0;
#pragma unroll
            for (int a0 = 0; a0 < PM; ++a0)
              if (a0 < p) t = fma(L[0][a0], yh[a0 + p * a1], t);
            s = fma(L[D - 1][a1], t, s);
          }
        }
      } else {
#pragma unroll
        for (int a2 = 0; a2 < PM; ++a2) {
          if (a2 < p) {
            double t2 = 0;
#pragma unroll
            for (int a1 = 0; a1 < PM; ++a1) {
              if (a1 < p) {
                double t = 0;
#pragma unroll
                for (int a0 = 0; a0 < PM; ++a0)
                  if (a0 < p) t = fma(L[0][a0], yh[a0 + p * (a1 + p * a2)], t);
                t2 = fma(L[1][a1], t, t2);
              }
            }
            s = fma(L[D - 1][a2], t2, s);
          }
        }
      }
      acc += s;
    }
  }
  wsum[w][i] = acc;
  __syncthreads();
  if (w == 0 && i < m) {
    double v = wsum[0][i] + wsum[1][i] + wsum[2][i] + wsum[3][i];
    v += near_partials(part, part_ptr[leaf], part_ptr[leaf + 1], part_idx, i);
    Y[perm[s0 + i]] = v;
  }
}


// ================================================= several columns (MFMA) ===
// FP64 matrix cores, v_mfma_f64_16x16x4f64.  Operand layout per lane l of a
// wavefront: A[l % 16][l / 16] (16 x 4), B[l / 16][l % 16] (4 x 16); the
// 16 x 16 result has D[(l / 16) + 4 r][l % 16] in register r.
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One column with stored couplings, grouped: item it covers rows
// [64 rb, 64 rb + 64) of the coupled coefficients of up to kGrpSlots
// targets that share one sequence of stored matrices K_e (K_e(b, a) at
// koff_e + b pd + a, the partner's nodes b as rows):
// y_c[a] = sum_e sum_b K_e(b, a) x_{t_e(c)}[b].  Lanes run over the rows a
// (coalesced reads of K), each entry K_e(b, a) read once serves every target
// of the item, and the partners' moments x_{t_e(c)}[b..b+7] are wave-uniform
// (scalar loads).  Wavefront w takes the sequence entries e = w, w + 8, ...;
// the eight partial sums are added in wavefront order through LDS (fixed
// order, deterministic).
template <typename KT>
__global__ void __launch_bounds__(512) k_couple_grp1(const GroupItem *__restrict__ items,
                                                     const int64_t *__restrict__ grp_koff,
                                                     const int32_t *__restrict__ grp_pdt,
                                                     const int32_t *__restrict__ grp_tcoef,
                                                     const int32_t *__restrict__ grp_xoff,
                                                     const KT *__restrict__ kst,
                                                     const double *__restrict__ xhat,
                                                     double *__restrict__ yhat) {
  constexpr int T = kGrpSlots;
  __shared__ double red[8][T][64];
  const GroupItem it = items[blockIdx.x];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
  const int a = 64 * it.rb + l;
  const bool aok = a < it.pd;
  const int ar = aok ? a : 0;
  double acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = 0.0;
  for (int e = w; e < it.len; e += 8) {
    const int pdt = grp_pdt[it.seq + e];
    const KT *K = kst + grp_koff[it.seq + e] + ar;
    const double *x[T];
#pragma unroll
    for (int t = 0; t < T; ++t)
      x[t] = xhat + grp_xoff[it.xbase + (t < it.nslot ? t : 0) * it.len + e];
    int b = 0;
    for (; b + 8 <= pdt; b += 8) {
      double k[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) k[u] = (double)K[(int64_t)(b + u) * it.pd];
#pragma unroll
      for (int t = 0; t < T; ++t)
        if (t < it.nslot) {
#pragma unroll
          for (int u = 0; u < 8; ++u) acc[t] = fma(k[u], x[t][b + u], acc[t]);
        }
    }
    for (; b < pdt; ++b) {
      const double k = (double)K[(int64_t)b * it.pd];
#pragma unroll
      for (int t = 0; t < T; ++t)
        if (t < it.nslot) acc[t] = fma(k, x[t][b], acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < T; ++t) red[w][t][l] = acc[t];
  __syncthreads();
  for (int e2 = threadIdx.x; e2 < T * 64; e2 += 512) {
    const int t = e2 >> 6, row = e2 & 63;
    const int ao = 64 * it.rb + row;
    if (t < it.nslot && ao < it.pd) {
      double v = red[0][t][row];
#pragma unroll
      for (int q = 1; q < 8; ++q) v += red[q][t][row];
      yhat[grp_tcoef[it.slot0 + t] + ao] = v;
    }
  }
}

// Upward pass, one column, two dimensions, on the FP64 matrix cores: for one
// chunk of <= kUpChunk points of a far cluster, Xhat[a0][a1] =
// sum_i L0_i[a0] (x_i L1_i[a1]) is a 16 x 16 product accumulated over the
// points four at a time (v_mfma_f64_16x16x4f64).  One wavefront per chunk;
// lane l evaluates the Lagrange values of point l of each 64-point block
// into LDS.
__global__ void __launch_bounds__(64) k_up1_mfma2(const UpItem *__restrict__ items,
                                                  const FarCluster *__restrict__ fc,
                                                  const double *__restrict__ pts, int64_t n,
                                                  const double *__restrict__ cheb,
                                                  const double *__restrict__ xt,
                                                  double *__restrict__ part_up) {
  __shared__ double L0s[64][17], L1s[64][17];
  const UpItem it = items[blockIdx.x];
  const FarCluster c = fc[it.fc];
  const int p = c.p;
  const int l = threadIdx.x, lr = l & 15, lk = l >> 4;
  const double *cu = cheb + p * 2 * kMaxCheb;
  v4d acc = {0, 0, 0, 0};
  for (int64_t i0 = it.begin; i0 < it.end; i0 += 64) {
    const int64_t i = i0 + l;
    double L0[16], L1[16];
    if (i < it.end) {
      const double x0 = pts[i], x1 = pts[n + i], xv = xt[i];
      lagrange_prod<16>(p, cu, cu + kMaxCheb, c.hw[0] > 0 ? (x0 - c.ctr[0]) / c.hw[0] : 0.0, L0);
      lagrange_prod<16>(p, cu, cu + kMaxCheb, c.hw[1] > 0 ? (x1 - c.ctr[1]) / c.hw[1] : 0.0, L1);
#pragma unroll
      for (int a = 0; a < 16; ++a) L1[a] *= xv;
    } else {
#pragma unroll
      for (int a = 0; a < 16; ++a) L0[a] = L1[a] = 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      L0s[l][a] = L0[a];
      L1s[l][a] = L1[a];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 4 * kk + lk;
      acc = mfma4(L0s[k][lr], L1s[k][lr], acc);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a0 = lk + 4 * r, a1 = lr;
    if (a0 < p && a1 < p) part_up[it.poff + a0 + p * a1] = acc[r];
  }
}

// Downward pass + near-field partials + scatter, one column, two dimensions:
// for every far ancestor c of the leaf, y_i += L0_i^T Yhat_c L1_i, formed as
// C = Yhat_c L1^T on the matrix cores (16 points per tile) and contracted
// with L0 per point.  Four waves split the ancestors; lane l owns point l.
__global__ void __launch_bounds__(256) k_final1_mfma2(
    const int64_t *__restrict__ leaf_off, const double *__restrict__ pts, int64_t n,
    const double *__restrict__ cheb, const FarCluster *__restrict__ fc,
    const int32_t *__restrict__ anc_ptr, const int32_t *__restrict__ anc_idx,
    const double *__restrict__ yhat, const double *__restrict__ part,
    const int32_t *__restrict__ part_ptr, const int32_t *__restrict__ part_idx,
    const int64_t *__restrict__ perm, double *__restrict__ Y) {
  __shared__ double L0s[4][64][17], L1s[4][64][17];
  __shared__ double wsum[4][64];
  const int leaf = blockIdx.x;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
  const int64_t s0 = leaf_off[leaf], m = leaf_off[leaf + 1] - s0;
  double x0 = 0, x1 = 0;
  if (l < m) {
    x0 = pts[s0 + l];
    x1 = pts[n + s0 + l];
  }
  double yacc = 0;
  for (int e = anc_ptr[leaf] + w; e < anc_ptr[leaf + 1]; e += 4) {
    const FarCluster c = fc[__builtin_amdgcn_readfirstlane(anc_idx[e])];
    const int p = c.p;
    const double *cu = cheb + p * 2 * kMaxCheb;
    const double *yh = yhat + c.coef_off;
    double L0[16], L1[16];
    if (l < m) {
      lagrange_prod<16>(p, cu, cu + kMaxCheb, c.hw[0] > 0 ? (x0 - c.ctr[0]) / c.hw[0] : 0.0, L0);
      lagrange_prod<16>(p, cu, cu + kMaxCheb, c.hw[1] > 0 ? (x1 - c.ctr[1]) / c.hw[1] : 0.0, L1);
    } else {
#pragma unroll
      for (int a = 0; a < 16; ++a) L0[a] = L1[a] = 0.0;
    }
    double yv[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int a0 = lr, a1 = 4 * kk + lk;
      yv[kk] = (a0 < p && a1 < p) ? yh[a0 + p * a1] : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      L0s[w][l][a] = L0[a];
      L1s[w][l][a] = L1[a];
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): LDS writes done
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {
      v4d acc = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc = mfma4(yv[kk], L1s[w][16 * jt + lr][4 * kk + lk], acc);
      double sv = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) sv = fma(L0s[w][16 * jt + lr][lk + 4 * r], acc[r], sv);
      sv += __shfl_xor(sv, 16);
      sv += __shfl_xor(sv, 32);
      if (lk == jt) yacc += sv;
    }
    __builtin_amdgcn_wave_barrier();
  }
  wsum[w][l] = yacc;
  __syncthreads();
  if (w == 0 && l < m) {
    double v = wsum[0][l] + wsum[1][l] + wsum[2][l] + wsum[3][l];
    v += near_partials(part, part_ptr[leaf], part_ptr[leaf + 1], part_idx, l);
    Y[perm[s0 + l]] = v;
  }
}


// Sum the chunk partials (pd x nrhs each) of every far cluster.
__global__ void __launch_bounds__(256) k_up_reduce_m(const FarCluster *__restrict__ fc,
                                                     const int32_t *__restrict__ item_ptr,
                                                     const UpItem *__restrict__ items, int nrhs,
                                                     const double *__restrict__ part,
                                                     double *__restrict__ xhat) {
  const FarCluster c = fc[blockIdx.x];
  const int i0 = item_ptr[blockIdx.x], i1 = item_ptr[blockIdx.x + 1];
  const int64_t tot = (int64_t)c.pd * nrhs;
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.y * 256) {
    double s = 0;
    for (int it = i0; it < i1; ++it) s += part[items[it].poff * nrhs + e];
    xhat[c.coef_off * nrhs + e] = s;
  }
}

// Lagrange values of every far cluster's points at its nodes, computed once
// at build: lag[lag_off + ((i - begin) * D + k) * PMax + a] = l_a(z_k(x_i)),
// zero for a >= p (one thread per point and axis of an upward chunk).
template <int D>
__global__ void __launch_bounds__(256) k_lagrange_table(const UpItem *__restrict__ items,
                                                        const FarCluster *__restrict__ fc,
                                                        const double *__restrict__ pts, int64_t n,
                                                        const double *__restrict__ cheb,
                                                        double *__restrict__ lag) {
  constexpr int PM = PMax<D>::v;
  const UpItem it = items[blockIdx.x];
  const int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x;
  const int64_t i = it.begin + e / D;
  const int k = (int)(e % D);
  if (i >= it.end) return;
  const FarCluster c = fc[it.fc];
  const double *cu = cheb + c.p * 2 * kMaxCheb;
  const double x = pts[k * n + i];
  const double hw = fc[it.fc].hw[k], ctr = fc[it.fc].ctr[k];
  const double z = hw > 0 ? (x - ctr) / hw : 0.0;
  double L[PM];
  lagrange_any<PM>(c.p, cu, cu + kMaxCheb, z, L);
  double *o = lag + c.lag_off + ((i - c.begin) * D + k) * PM;
#pragma unroll
  for (int a = 0; a < PM; ++a) o[a] = L[a];
}

// Upward pass of the several-column product: the partial U_c^T X of one
// chunk of cluster c's points, for one 64-row block of its coefficients and
// 512 columns per workgroup.  Per 16 points: the per-axis Lagrange values go
// to LDS, the workgroup forms the 64 x 16 block of basis values once
// (double-buffered in LDS), and wavefront w multiplies it with columns
// [64 w, 64 w + 64) of X read straight from global memory one chunk ahead.
template <int D>
__global__ void __launch_bounds__(512) k_up_mfma2(const CoupleMItem *__restrict__ blocks,
                                                  const UpItem *__restrict__ items,
                                                  const FarCluster *__restrict__ fc,
                                                  const double *__restrict__ lag, int64_t n,
                                                  const double *__restrict__ xt, int nrhs,
                                                  double *__restrict__ part) {
  constexpr int PM = PMax<D>::v, LDK = 18;
  __shared__ double Ls[D][16][PM + 1];
  __shared__ double As[2][64 * LDK];
  const CoupleMItem bk = blocks[blockIdx.x];
  const UpItem it = items[bk.s];
  const FarCluster c = fc[it.fc];
  const int p = c.p, pd = c.pd;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int lr = l & 15, lk = l >> 4;
  const int r0 = 64 * bk.rb;
  const int rows = min(64, pd - r0);
  const int nrb = (rows + 15) >> 4;
  const int c0 = blockIdx.y * 512 + 64 * w;
  // 16-column blocks of this wavefront inside nrhs (wave-uniform)
  const int ncb = min(4, max(0, (nrhs - c0 + 15) >> 4));
  // basis role: row er, points ek, ek + 1 of a chunk
  const int er = tid >> 3, ek = 2 * (tid & 7);
  int dig[D];
  {
    int r = er < rows ? r0 + er : 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      dig[k] = r % p;
      r /= p;
    }
  }
  auto load_b = [&](int64_t i0, double *b) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int64_t i = i0 + 4 * kk + lk;
      const int64_t ic = i < it.end ? i : it.begin;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int cc = c0 + 16 * j + lr;
        b[4 * kk + j] = xt[ic + n * (int64_t)(cc < nrhs ? cc : 0)];
      }
    }
  };
  v4d acc[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[q][j] = v4d{0, 0, 0, 0};
  double bcur[16], bnext[16];
  int buf = 0;
  load_b(it.begin, bcur);
  for (int64_t i0 = it.begin; i0 < it.end; i0 += 16) {
    {
      // one (axis, point, node) per thread, from the table built with the
      // operator
      const int a = tid % PM, i = (tid / PM) & 15, k = tid / (PM * 16);
      if (k < D)
        Ls[k][i][a] = i0 + i < it.end ? lag[c.lag_off + ((i0 + i - c.begin) * D + k) * PM + a]
                                      : 0.0;
    }
    if (i0 + 16 < it.end) load_b(i0 + 16, bnext);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double v = Ls[0][ek + h][dig[0]];
#pragma unroll
      for (int k = 1; k < D; ++k) v *= Ls[k][ek + h][dig[k]];
      As[buf][er * LDK + ek + h] = er < rows ? v : 0.0;
    }
    __syncthreads();
    const double *A = As[buf];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < nrb) {
          const double a = A[(16 * q + lr) * LDK + 4 * kk + lk];
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (j < ncb) acc[q][j] = mfma4(a, bcur[4 * kk + j], acc[q][j]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) bcur[i] = bnext[i];
    buf ^= 1;
  }
  double *o = part + it.poff * nrhs;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * q + lk + 4 * r;
        const int cc = c0 + 16 * j + lr;
        if (a < rows && cc < nrhs) o[r0 + a + (int64_t)pd * cc] = acc[q][j][r];
      }
}

// Workgroups are dealt to the eight XCDs in turn (linear workgroup id mod
// 8).  xcd_contiguous maps workgroup b of n so that each XCD's workgroups
// cover one contiguous range of indices, e.g. of leaves, whose shared
// ancestors' data then stays in that XCD's L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
  const int x = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
  return x * q + min(x, r) + k;
}

// Downward pass of the several-column product: Y[perm, c] += U_c|_s Yhat_c
// over the far ancestors c of leaf s, for 256 columns per workgroup.  Per
// ancestor the per-axis Lagrange values of the leaf's points go to LDS; per
// 16 coefficients the workgroup forms the 64 x 16 block of basis values once
// (double-buffered in LDS), and wavefront w multiplies it with columns
// [32 w, 32 w + 32) of Yhat_c read straight from global memory one chunk
// ahead.  (A 64 x 32 tile per wavefront keeps it within 128 registers, so
// two workgroups share a CU and one's matrix-core work covers the other's
// barriers: 13 % faster than 64 x 64 tiles with one workgroup per CU.)
template <int D>
__global__ void __launch_bounds__(512, 2) k_down_mfma2(
    const int64_t *__restrict__ leaf_off, const double *__restrict__ pts, int64_t n,
    const double *__restrict__ cheb, const FarCluster *__restrict__ fc,
    const int32_t *__restrict__ anc_ptr, const int32_t *__restrict__ anc_idx,
    const double *__restrict__ yhat, const int32_t *__restrict__ ynz,
    const int64_t *__restrict__ perm, int nrhs, const int32_t *__restrict__ ocol, int ocol0,
    double *__restrict__ Y, int64_t ldy) {
  constexpr int PM = PMax<D>::v, LDK = 18;
  __shared__ double Ls[D][64][PM + 1];
  __shared__ double As[2][64 * LDK];
  const int s = xcd_contiguous(blockIdx.x, gridDim.x);   // leaves of a subtree on one XCD
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int lr = l & 15, lk = l >> 4;
  const int64_t s0 = leaf_off[s], ms = leaf_off[s + 1] - s0;
  const int nrb = (int)((ms + 15) >> 4);
  const int c0 = blockIdx.y * 256 + 32 * w;
  // 16-column blocks of this wavefront inside nrhs (wave-uniform)
  const int ncb = min(2, max(0, (nrhs - c0 + 15) >> 4));
  const int er = tid >> 3, ek = 2 * (tid & 7);   // basis role: point er, coefficients ek, ek+1
  const int ea = anc_ptr[s], eb = anc_ptr[s + 1];
  // with ynz (nonzero 16-column blocks of each cluster's Yhat): bit j of the
  // wave-uniform mask is set when block j of this wavefront is nonzero for
  // ancestor e; zero blocks are neither loaded nor multiplied
  const int ncb16 = (nrhs + 15) >> 4;
  auto nz_mask = [&](int e) -> int {
    if (!ynz) return 3;
    const int32_t *f = ynz + (int64_t)anc_idx[e] * ncb16 + (c0 >> 4);
    int m = 0;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (j < ncb && f[j]) m |= 1 << j;
    return __builtin_amdgcn_readfirstlane(m);
  };
  auto load_b = [&](int e, int a0, int msk, double *b) {
    const FarCluster c = fc[anc_idx[e]];
    const double *y = yhat + c.coef_off * nrhs;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int a = a0 + 4 * kk + lk;
      const int ac = a < c.pd ? a : 0;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int cc = c0 + 16 * j + lr;
        b[2 * kk + j] = (msk >> j & 1) ? y[ac + (int64_t)c.pd * (cc < nrhs ? cc : 0)] : 0.0;
      }
    }
  };
  v4d acc[4][2];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[q][j] = v4d{0, 0, 0, 0};
  double bcur[8], bnext[8];
  int buf = 0;
  int e = ea, a0 = 0;
  int mcur = e < eb ? nz_mask(e) : 0, mnext = mcur;
  if (e < eb) load_b(e, 0, mcur, bcur);
  while (e < eb) {
    const int ci = anc_idx[e];
    const int p = fc[ci].p, pd = fc[ci].pd;
    const double *cu = cheb + p * 2 * kMaxCheb;
    if (a0 == 0 && tid < D * 64) {
      // Lagrange values of (axis k, point i) at the ancestor's nodes:
      // l_a(z) = (w_a / (z - u_a)) / sum_m w_m / (z - u_m)
      const int i = tid & 63, k = tid >> 6;
      if (i < ms) {
        const double x = pts[k * n + s0 + i];
        const double hw = fc[ci].hw[k], ctr = fc[ci].ctr[k];
        const double z = hw > 0 ? (x - ctr) / hw : 0.0;
        double sum = 0.0;
        int exact = -1;
        for (int m = 0; m < p; ++m) {
          const double dx = z - cu[m];
          if (dx == 0.0) exact = m;
          sum += cu[kMaxCheb + m] * rcp_nr(dx == 0.0 ? 1.0 : dx);
        }
        const double is = rcp_nr(sum);
        for (int m = 0; m < PM; ++m) {
          double v = 0.0;
          if (m < p) {
            const double dx = z - cu[m];
            v = exact >= 0 ? (m == exact ? 1.0 : 0.0)
                           : cu[kMaxCheb + m] * rcp_nr(dx == 0.0 ? 1.0 : dx) * is;
          }
          Ls[k][i][m] = v;
        }
      } else {
        for (int m = 0; m < PM; ++m) Ls[k][i][m] = 0.0;
      }
    }
    // next chunk
    int en = e, an = a0 + 16;
    if (an >= pd) {
      ++en;
      an = 0;
      if (en < eb) mnext = nz_mask(en);
    }
    if (en < eb) load_b(en, an, mnext, bnext);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int a = a0 + ek + h;
      double v = 0.0;
      if (a < pd) {
        v = Ls[0][er][a % p];
        a /= p;
#pragma unroll
        for (int k = 1; k < D; ++k) {
          v *= Ls[k][er][a % p];
          a /= p;
        }
      }
      As[buf][er * LDK + ek + h] = v;
    }
    __syncthreads();
    const double *A = As[buf];
    // k-steps past the ancestor's pd multiply zeros: skipped
    const int nkk = min(4, (pd - a0 + 3) >> 2);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      if (kk >= nkk) break;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < nrb) {
          const double av = A[(16 * q + lr) * LDK + 4 * kk + lk];
#pragma unroll
          for (int j = 0; j < 2; ++j)
            if (j < ncb && (mcur >> j & 1)) acc[q][j] = mfma4(av, bcur[2 * kk + j], acc[q][j]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) bcur[i] = bnext[i];
    mcur = mnext;
    buf ^= 1;
    e = en;
    a0 = an;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * q + lk + 4 * r;
        const int cc = c0 + 16 * j + lr;
        if (i < ms && cc < nrhs) {
          const int oc = ocol ? ocol[ocol0 + cc] : ocol0 + cc;
          double *y = Y + perm[s0 + i] + ldy * oc;
          *y += acc[q][j][r];
        }
      }
}

__global__ void k_zero(double *__restrict__ p, int64_t len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) p[i] = 0.0;
}

// Couplings of the several-column product, Yhat_s = sum over admissible t of
// K(xi_s, xi_t) Xhat_t, for one 64-row block of cluster s and 256 columns per
// workgroup.  Each 64 x 16 chunk of K goes to LDS once per workgroup
// (double-buffered, one barrier per chunk): read from the pair's stored
// matrix one chunk ahead where the couplings are stored (ST), else evaluated;
// wavefront w multiplies it with columns [32 w, 32 w + 32) of Xhat_t, whose B
// operands it reads straight from global memory one chunk ahead (every
// 32-byte sector fully used).  Rows past the cluster and coefficients past
// the partner are zero in K; only the 16-row blocks inside the cluster are
// multiplied.  (Reading the stored matrices instead of evaluating K: 2.20 ->
// 1.49 ms on the 480-ray crosswell; 64 x 32 tiles instead of 64 x 64, with two
// workgroups per CU: 1.49 -> 1.34 ms.)
template <int D, bool F32, bool ST>
__global__ void __launch_bounds__(512, 2) k_couple_mfma2(
    const CoupleMItem *__restrict__ items, const FarCluster *__restrict__ fc,
    const int32_t *__restrict__ far_ptr, const int32_t *__restrict__ far_col,
    const double *__restrict__ cheb, int kind, double inv_ell, double amp,
    const int64_t *__restrict__ far_koff, const void *__restrict__ kst_v,
    const double *__restrict__ xhat, int nrhs, double *__restrict__ yhat,
    const int32_t *__restrict__ nzb, const int32_t *__restrict__ plist,
    const int32_t *__restrict__ pcnt) {
  typedef typename std::conditional<F32, float, double>::type KT;
  const KT *__restrict__ kst = reinterpret_cast<const KT *>(kst_v);
  constexpr int KC = 16, LDK = 18;
  __shared__ double Ks[2][64 * LDK];
  const CoupleMItem it = items[blockIdx.x];
  const FarCluster cs = fc[it.s];
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int lr = l & 15, lk = l >> 4;
  const int r0 = 64 * it.rb;
  const int rows = min(64, cs.pd - r0);
  const int nrb = (rows + 15) >> 4;
  const int c0 = blockIdx.y * 256 + 32 * w;
  // 16-column blocks of this wavefront inside nrhs (wave-uniform)
  const int ncb = min(2, max(0, (nrhs - c0 + 15) >> 4));
  const double scale = kernel_c(kind) * inv_ell;
  // K evaluation role of this thread: row er, chunk columns ek, ek + 1
  const int er = tid >> 3, ek = 2 * (tid & 7);
  double xs[D];
  if (!ST) {
    int r = er < rows ? r0 + er : 0;
    const double *us = cheb + cs.p * 2 * kMaxCheb;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      xs[k] = scale * (cs.ctr[k] + cs.hw[k] * us[r % cs.p]);
      r /= cs.p;
    }
  }
  // partners: the far list of it.s, or (plist) those of its partners whose
  // moments are nonzero somewhere in this workgroup's 256 columns; chunk
  // sequence: (partner index e, first coefficient k0), far-list entry E(e)
  int e0 = far_ptr[it.s], e1 = far_ptr[it.s + 1];
  const int32_t *pl = nullptr;
  if (plist) {
    pl = plist + (int64_t)e0 * gridDim.y + (int64_t)blockIdx.y * (e1 - e0);
    e1 = pcnt[(int64_t)it.s * gridDim.y + blockIdx.y];
    e0 = 0;
  }
  auto E = [&](int e) { return pl ? pl[e] : e; };
  auto eval_chunk = [&](int e, int k0, int buf) {
    const FarCluster ct = fc[far_col[E(e)]];
    const double *ut = cheb + ct.p * 2 * kMaxCheb;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kb = k0 + ek + h;
      int r = kb < ct.pd ? kb : 0;
      double t2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double dx = xs[k] - scale * (ct.ctr[k] + ct.hw[k] * ut[r % ct.p]);
        t2 = fma(dx, dx, t2);
        r /= ct.p;
      }
      const double kv = kernel_t2<F32>(t2, kind, amp);
      Ks[buf][er * LDK + ek + h] = (er < rows && kb < ct.pd) ? kv : 0.0;
    }
  };
  // stored couplings (ST): this thread's two entries of a chunk, read from
  // the pair's matrix (column-major, leading dimension pd of the target)
  // one chunk ahead and put in LDS at the top of the chunk
  auto load_k = [&](int e, int k0, double *kv) {
    const KT *K = kst + far_koff[E(e)];
    const int pdt = fc[far_col[E(e)]].pd;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kb = k0 + ek + h;
      kv[h] = (er < rows && kb < pdt) ? (double)K[(r0 + er) + (int64_t)kb * cs.pd] : 0.0;
    }
  };
  // with nzb (moments of sparse columns: nzb[t ncb16 + b] = 0 when the
  // 16-column block b of partner t's coefficients is exactly zero): bit j of
  // the wave-uniform mask is set when block j of this wavefront is nonzero;
  // zero blocks are not multiplied (their products would add zeros)
  const int ncb16 = (nrhs + 15) >> 4;
  auto nz_mask = [&](int e) -> int {
    if (!nzb) return 3;
    const int32_t *f = nzb + (int64_t)far_col[E(e)] * ncb16 + (c0 >> 4);
    int m = 0;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (j < ncb && f[j]) m |= 1 << j;
    return __builtin_amdgcn_readfirstlane(m);
  };
  // B operands of a chunk; blocks that the mask marks zero are not loaded
  auto load_b = [&](int e, int k0, int msk, double *b) {
    const FarCluster ct = fc[far_col[E(e)]];
    const double *x = xhat + ct.coef_off * nrhs;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int kb = k0 + 4 * kk + lk;
      const int kc = kb < ct.pd ? kb : 0;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int c = c0 + 16 * j + lr;
        b[2 * kk + j] = (msk >> j & 1) ? x[kc + (int64_t)ct.pd * (c < nrhs ? c : 0)] : 0.0;
      }
    }
  };
  v4d acc[4][2];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[q][j] = v4d{0, 0, 0, 0};
  double bcur[8], bnext[8], kcur[2] = {0.0, 0.0}, knext[2] = {0.0, 0.0};
  int e = e0, k0 = 0, buf = 0;
  int mcur = e < e1 ? nz_mask(e) : 0, mnext = mcur;
  int pdc = e < e1 ? fc[far_col[E(e)]].pd : 0, pdn = pdc;   // partner pd of the chunk
  int mor = 0;   // blocks nonzero for some partner (the others of Yhat stay zero)
  if (e < e1) {
    load_b(e, k0, mcur, bcur);
    if (ST) load_k(e, k0, kcur);
  }
  while (e < e1) {
    if (ST) {
      Ks[buf][er * LDK + ek] = kcur[0];
      Ks[buf][er * LDK + ek + 1] = kcur[1];
    } else {
      eval_chunk(e, k0, buf);
    }
    // next chunk
    int en = e, kn = k0 + KC;
    if (kn >= pdc) {
      ++en;
      kn = 0;
      if (en < e1) {
        mnext = nz_mask(en);
        pdn = fc[far_col[E(en)]].pd;
      }
    }
    if (en < e1) {
      load_b(en, kn, mnext, bnext);
      if (ST) load_k(en, kn, knext);
    }
    __syncthreads();
    const double *K = Ks[buf];
    // k-steps past the partner's pd multiply zeros: skipped
    const int nkk = min(4, (pdc - k0 + 3) >> 2);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      if (kk >= nkk) break;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < nrb) {
          const double a = K[(16 * q + lr) * LDK + 4 * kk + lk];
#pragma unroll
          for (int j = 0; j < 2; ++j)
            if (j < ncb && (mcur >> j & 1)) acc[q][j] = mfma4(a, bcur[2 * kk + j], acc[q][j]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) bcur[i] = bnext[i];
    kcur[0] = knext[0];
    kcur[1] = knext[1];
    mor |= mcur;
    e = en;
    k0 = kn;
    mcur = mnext;
    pdc = pdn;
    buf ^= 1;
  }
  // with sparse moments a zero block of Yhat is not written (the downward
  // pass skips it by the same mask)
  if (!nzb) mor = 3;
  double *o = yhat + cs.coef_off * nrhs;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * q + lk + 4 * r;
        const int cc = c0 + 16 * j + lr;
        if (a < rows && cc < nrhs && (mor >> j & 1)) o[r0 + a + (int64_t)cs.pd * cc] = acc[q][j][r];
      }
}

// Tiles of the ordered near pairs in MFMA operand order.  Pair e (entry e of
// near_idx: stored tile b, used as is or transposed) becomes 4096 entries
// frag[e][w][kk][l] = A[16 w + l % 16][4 kk + l / 16] with A = tile or
// tile^T: the A operand of step kk of the 16 x 16 x 4 FP64 MFMA for rows
// 16w..16w+15, so that a wavefront loads its operands with coalesced
// 64-lane loads.  One workgroup per ordered pair.
template <typename TT>
__global__ void __launch_bounds__(256) k_near_repack(const TT *__restrict__ blk,
                                                     const int32_t *__restrict__ near_idx,
                                                     TT *__restrict__ frag) {
  __shared__ double As[64][65];
  const int64_t e = blockIdx.x;
  const int code = near_idx[e];
  const int64_t b = code >> 1;
  const bool trans = code & 1;
  const int tid = threadIdx.x;
  if (sizeof(TT) == 8) {
    const v2d *src = reinterpret_cast<const v2d *>(blk + b * 4096);
    for (int q = tid; q < 2048; q += 256) {
      const int k = q >> 6, lane = q & 63;
      const int i = 8 * (lane & 7) + (k >> 2), j = 8 * (lane >> 3) + 2 * (k & 3);
      const v2d v = src[q];
      if (!trans) {
        As[i][j] = v.x;
        As[i][j + 1] = v.y;
      } else {
        As[j][i] = v.x;
        As[j + 1][i] = v.y;
      }
    }
  } else {
    const float4 *src = reinterpret_cast<const float4 *>(blk + b * 4096);
    for (int q = tid; q < 1024; q += 256) {
      const int k = q >> 6, lane = q & 63;
      const int i = 8 * (lane & 7) + (k >> 1), j = 8 * (lane >> 3) + 4 * (k & 1);
      const float4 v = src[q];
      const double vv[4] = {v.x, v.y, v.z, v.w};
      for (int h = 0; h < 4; ++h) {
        if (!trans)
          As[i][j + h] = vv[h];
        else
          As[j + h][i] = vv[h];
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < 4096; idx += 256) {
    const int w = idx >> 10, kk = (idx >> 6) & 15, l = idx & 63;
    frag[e * 4096 + idx] = (TT)As[16 * w + (l & 15)][4 * kk + (l >> 4)];
  }
}

// Near field of the several-column product on the FP64 matrix cores,
// Y[perm, c] = sum over the near pairs (s, t) of A_st X_t: one workgroup per
// (target leaf s, block of 128 columns), eight wavefronts, each owning 16 rows
// and 64 columns.  The A operands come from the repacked tiles straight into
// registers (coalesced, one pair ahead); the 64 x 128 block of X_t goes
// through LDS, stored column-major with row stride 66 (conflict-free operand
// reads) and double-buffered, so that a pair costs one barrier.  Rows of X_t beyond the
// leaf and columns beyond nrhs are staged as zeros.
template <typename TT>
__global__ void __launch_bounds__(512) k_near_mfma(
    const TT *__restrict__ frag, const int32_t *__restrict__ near_ptr,
    const int32_t *__restrict__ near_idx, const int32_t *__restrict__ bs,
    const int32_t *__restrict__ bt, const int64_t *__restrict__ leaf_off, int64_t n,
    const double *__restrict__ xt, const int64_t *__restrict__ perm, int nrhs,
    double *__restrict__ Y, int64_t ldy) {
  constexpr int NC = 128, LDB = 66;
  __shared__ double Bt[2][NC * LDB];
  const int s = blockIdx.x;
  const int c0 = blockIdx.y * NC;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int rg = w & 3, ch = w >> 2;   // 16-row group and 64-column half of this wavefront
  const int lr = l & 15, lk = l >> 4;
  const int e0 = near_ptr[s], e1 = near_ptr[s + 1];
  const int64_t s0 = leaf_off[s], ms = leaf_off[s + 1] - s0;
  double breg[16], acur[16], anext[16];
  // X_t block of pair e into registers: thread (k = l, columns w + 8q)
  auto load_b = [&](int e) {
    const int code = near_idx[e];
    const int64_t b = code >> 1;
    const int t = (code & 1) ? bs[b] : bt[b];
    const int64_t t0 = leaf_off[t], mt = leaf_off[t + 1] - t0;
    const bool row_ok = l < mt;
    const int64_t r = t0 + (row_ok ? l : 0);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = c0 + w + 8 * q;
      const double v = xt[r + n * (int64_t)(c < nrhs ? c : 0)];
      breg[q] = (row_ok && c < nrhs) ? v : 0.0;
    }
  };
  auto store_b = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 16; ++q) Bt[buf][(w + 8 * q) * LDB + l] = breg[q];
  };
  auto load_a = [&](int e, double *a) {
    const TT *src = frag + (int64_t)e * 4096 + rg * 1024 + l;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) a[kk] = (double)src[kk * 64];
  };
  v4d acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = v4d{0, 0, 0, 0};
  if (e1 > e0) {   // (every leaf is near itself; kept for safety)
    load_b(e0);
    load_a(e0, acur);
    store_b(0);
  }
  __syncthreads();
  for (int e = e0; e < e1; ++e) {
    const int cur = (e - e0) & 1;
    const bool more = e + 1 < e1;
    if (more) {
      load_b(e + 1);
      load_a(e + 1, anext);
    }
    const double *B = Bt[cur] + (64 * ch) * LDB;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 4 * kk + lk;
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = mfma4(acur[kk], B[(16 * j + lr) * LDB + k], acc[j]);
    }
    if (more) {
      store_b(cur ^ 1);
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) acur[kk] = anext[kk];
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = rg * 16 + lk + 4 * r;
      const int cc = c0 + 64 * ch + j * 16 + lr;
      if (i < ms && cc < nrhs) Y[perm[s0 + i] + ldy * cc] = acc[j][r];
    }
}

}  // namespace fkf

// ------------------------------------------------------------------ host ---
using namespace fkf;

namespace {

// Stored coupling matrices are shared by pairs of the same geometry:
// K(xi_s, xi_t) depends on a pair of boxes only through the node counts, the
// half-widths and the offset of the two box centres.  coupling_quantum gives
// the scale that maps lengths to integers of 2^-40 of the extent of the
// boxes; coupling_key the key of the pair (a, b) with p_a, p_b nodes per
// dimension.  Pairs with equal keys point at one stored matrix.
double coupling_quantum(int d, const std::vector<const double *> &ctr,
                        const std::vector<const double *> &hw) {
  double ext = 0.0;
  for (int k = 0; k < d; ++k) {
    double lo = INFINITY, hi = -INFINITY;
    for (size_t c = 0; c < ctr.size(); ++c) {
      lo = std::min(lo, ctr[c][k] - hw[c][k]);
      hi = std::max(hi, ctr[c][k] + hw[c][k]);
    }
    ext = std::max(ext, hi - lo);
  }
  return ext > 0 ? std::ldexp(1.0, 40) / ext : 0.0;
}

std::vector<int64_t> coupling_key(int d, int pa, int pb, const double *ca, const double *ha,
                                  const double *cb, const double *hb, double q) {
  std::vector<int64_t> key{pa, pb};
  for (int k = 0; k < d; ++k) {
    key.push_back(std::llround((ca[k] - cb[k]) * q));
    key.push_back(std::llround(ha[k] * q));
    key.push_back(std::llround(hb[k] * q));
  }
  return key;
}

}  // namespace

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
    FKF_REQUIRE(kp->kind >= 0 && kp->kind <= 5, "fkf_cov_build: unknown kernel kind");
    FKF_REQUIRE(kp->variance > 0 && kp->length > 0, "fkf_cov_build: variance and length must be > 0");
    FKF_REQUIRE(hp->leaf_size >= 1 && hp->leaf_size <= kTile, "fkf_cov_build: leaf_size in 1..64");
    FKF_REQUIRE(hp->cheb_order >= 2 && hp->cheb_order <= kMaxCheb, "fkf_cov_build: cheb_order in 2..16");
    FKF_REQUIRE(hp->block_tol <= 0 || (hp->cheb_order_max >= hp->cheb_order &&
                                       hp->cheb_order_max <= kMaxCheb),
                "fkf_cov_build: cheb_order_max in cheb_order..16");
    FKF_REQUIRE(hp->eta > 0, "fkf_cov_build: eta must be > 0");
    FKF_REQUIRE(hp->precision == FKF_FP64 || hp->precision == FKF_MIXED,
                "fkf_cov_build: unknown precision");
    FKF_REQUIRE(hp->far_eval == 0 || hp->far_eval == 1, "fkf_cov_build: far_eval must be 0 or 1");
    FKF_REQUIRE(hp->workspace_bytes >= 0, "fkf_cov_build: workspace_bytes < 0");
    for (int64_t i = 0; i < n * d; ++i)
      FKF_REQUIRE(std::isfinite(pts_host[i]), "fkf_cov_build: non-finite coordinate");
    hipStream_t st = as_stream(stream);

    auto cov = std::make_unique<fkf_cov>();
    cov->n = n;
    cov->d = d;
    cov->kind = kp->kind;
    cov->theta = kp->variance;
    cov->ell = kp->length;
    cov->amp = kp->kind >= FKF_MATERN_12_DLENGTH ? kp->variance / kp->length : kp->variance;
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
    {
      // source leaf of every ordered near pair (near_idx order)
      std::vector<int32_t> nsrc(ni.size());
      for (size_t e = 0; e < ni.size(); ++e) {
        const int64_t b = ni[e] >> 1;
        nsrc[e] = (ni[e] & 1) ? bs2[b] : bt2[b];
      }
      cov->near_src.upload(nsrc, st);
      FKF_CHECK_HIP(hipStreamSynchronize(st));   // nsrc is a host temporary
    }
    cov->mixed = hp->precision == FKF_MIXED;
    if (cov->mixed) {
      cov->blk32.alloc((size_t)cov->n_blk * 4096);
      if (cov->n_blk > 0)
        hipLaunchKernelGGL(k_near_assemble32, dim3((unsigned)cov->n_blk), dim3(64), 0, st,
                           cov->pts.p, n, d, cov->leaf_off.p, cov->blk_s.p, cov->blk_t.p,
                           cov->kind, 1.0 / cov->ell, cov->amp, cov->blk32.p);
    } else {
      cov->blk.alloc((size_t)cov->n_blk * 4096);
      if (cov->n_blk > 0)
        hipLaunchKernelGGL(k_near_assemble, dim3((unsigned)cov->n_blk), dim3(64), 0, st,
                           cov->pts.p, n, d, cov->leaf_off.p, cov->blk_s.p, cov->blk_t.p,
                           cov->kind, 1.0 / cov->ell, cov->amp, cov->blk.p);
    }
    FKF_CHECK_HIP(hipGetLastError());
    if (cov->n_near_pairs > 0) {
      if (cov->mixed) {
        cov->frag32.alloc((size_t)cov->n_near_pairs * 4096);
        hipLaunchKernelGGL(k_near_repack<float>, dim3((unsigned)cov->n_near_pairs), dim3(256), 0,
                           st, cov->blk32.p, cov->near_idx.p, cov->frag32.p);
      } else {
        cov->frag.alloc((size_t)cov->n_near_pairs * 4096);
        hipLaunchKernelGGL(k_near_repack<double>, dim3((unsigned)cov->n_near_pairs), dim3(256), 0,
                           st, cov->blk.p, cov->near_idx.p, cov->frag.p);
      }
      FKF_CHECK_HIP(hipGetLastError());
    }

    // far clusters
    std::vector<int> fidx(t.nodes.size(), -1);
    std::vector<FarCluster> fcs;
    std::vector<PairItem> prs;     // unordered admissible pairs
    std::vector<CoupleItem> cis;   // their coupling sub-blocks
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
    // far clusters numbered in order of first appearance in the pair list
    // (first member before second); the plan numbers them the same way
    std::vector<std::pair<int, int>> fpairs;
    for (auto &pr : far) {
      const int a = far_id(pr.first);
      const int b = far_id(pr.second);
      fpairs.emplace_back(a, b);
    }
    cov->n_fc = (int)fcs.size();
    int64_t off = 0;
    int64_t lag_total = 0;
    const int pmax_d = d == 2 ? PMax<2>::v : PMax<3>::v;
    for (auto &c : fcs) {
      c.coef_off = off;
      off += c.pd;
      cov->max_pd = std::max(cov->max_pd, c.pd);
      c.lag_off = lag_total;
      lag_total += (c.end - c.begin) * d * pmax_d;
    }
    cov->n_coef = off;
    cov->n_interp = 0;
    for (auto &c : fcs) cov->n_interp += (c.end - c.begin) * (int64_t)c.pd;
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
    {
      // leaf range of every far cluster and the tree position of every point
      // (the sparse right-hand sides of the several-column product)
      std::vector<int32_t> fl(2 * fcs.size());
      bool ok = n <= (int64_t)INT32_MAX;
      for (size_t c = 0; c < fcs.size() && ok; ++c) {
        auto b = std::lower_bound(loff.begin(), loff.end(), fcs[c].begin);
        auto e = std::lower_bound(loff.begin(), loff.end(), fcs[c].end);
        ok = b != loff.end() && e != loff.end() && *b == fcs[c].begin && *e == fcs[c].end;
        fl[2 * c] = (int32_t)(b - loff.begin());
        fl[2 * c + 1] = (int32_t)(e - loff.begin());
      }
      if (ok && !fcs.empty()) {
        std::vector<int32_t> ip(n);
        for (int64_t i = 0; i < n; ++i) ip[t.perm[i]] = (int32_t)i;
        cov->fc_leaf.upload(fl, st);
        cov->iperm.upload(ip, st);
        FKF_CHECK_HIP(hipStreamSynchronize(st));   // fl, ip are host temporaries
        cov->sp_ok = true;
      }
    }
    cov->far_ptr.upload(fp, st);
    cov->far_col.upload(fcol, st);
    {
      // several-column coupling blocks: (cluster, 64-row block), ordered by
      // decreasing work (rows x sum of the partners' coefficients).  (Dealing
      // them to the eight XCDs level by level in spatial runs, so that an
      // XCD's items share partners, measured 10 % slower than this order;
      // keeping a cluster's row blocks on one XCD, no faster.)
      std::vector<std::pair<int64_t, CoupleMItem>> cm;
      for (int s = 0; s < cov->n_fc; ++s) {
        int64_t kext = 0;
        for (int e = fp[s]; e < fp[s + 1]; ++e) kext += fcs[fcol[e]].pd;
        if (kext == 0) {
          cov->cm_all = false;
          continue;
        }
        for (int rb = 0; 64 * rb < fcs[s].pd; ++rb) {
          const int rows = std::min(64, fcs[s].pd - 64 * rb);
          cm.push_back({(int64_t)rows * kext, CoupleMItem{s, rb}});
        }
      }
      std::stable_sort(cm.begin(), cm.end(),
                       [](const auto &a, const auto &b) { return a.first > b.first; });
      std::vector<CoupleMItem> cmi(cm.size());
      for (size_t i = 0; i < cm.size(); ++i) cmi[i] = cm[i].second;
      cov->n_cm_items = (int64_t)cmi.size();
      cov->cm_items.upload(cmi, st);
    }
    cov->anc_ptr.upload(ap, st);
    cov->anc_idx.upload(ai, st);
    // one-column work lists: upward chunks and unordered pairs
    {
      std::vector<UpItem> ups;
      std::vector<int32_t> uptr(1, 0);
      int64_t poff = 0;
      for (int c = 0; c < cov->n_fc; ++c) {
        for (int64_t b = fcs[c].begin; b < fcs[c].end; b += kUpChunk) {
          UpItem u{};
          u.fc = c;
          u.begin = b;
          u.end = std::min(b + kUpChunk, fcs[c].end);
          u.poff = poff;
          poff += fcs[c].pd;
          ups.push_back(u);
        }
        uptr.push_back((int32_t)ups.size());
      }
      cov->n_up_items = (int64_t)ups.size();
      cov->n_part_up = poff;
      cov->up_items.upload(ups, st);
      cov->up_ptr.upload(uptr, st);
      std::vector<UpItem> upm;
      std::vector<int32_t> uptrm(1, 0);
      int64_t poffm = 0;
      for (int c = 0; c < cov->n_fc; ++c) {
        for (int64_t b = fcs[c].begin; b < fcs[c].end; b += kUpChunkM) {
          UpItem u{};
          u.fc = c;
          u.begin = b;
          u.end = std::min(b + kUpChunkM, fcs[c].end);
          u.poff = poffm;
          poffm += fcs[c].pd;
          upm.push_back(u);
        }
        uptrm.push_back((int32_t)upm.size());
      }
      cov->n_up_items_m = (int64_t)upm.size();
      cov->n_part_up_m = poffm;
      cov->up_items_m.upload(upm, st);
      cov->up_ptr_m.upload(uptrm, st);
      cov->lag.alloc((size_t)std::max<int64_t>(lag_total, 1));
      {
        std::vector<std::pair<int64_t, CoupleMItem>> ub;
        for (size_t u = 0; u < upm.size(); ++u) {
          const int pd = fcs[upm[u].fc].pd;
          for (int rb = 0; 64 * rb < pd; ++rb)
            ub.push_back({(int64_t)std::min(64, pd - 64 * rb) * (upm[u].end - upm[u].begin),
                          CoupleMItem{(int32_t)u, rb}});
        }
        std::stable_sort(ub.begin(), ub.end(),
                         [](const auto &a, const auto &b) { return a.first > b.first; });
        std::vector<CoupleMItem> ubi(ub.size());
        for (size_t i = 0; i < ub.size(); ++i) ubi[i] = ub[i].second;
        cov->n_up_blocks_m = (int64_t)ubi.size();
        cov->up_blocks_m.upload(ubi, st);
      }
      std::vector<std::vector<int64_t>> cpl(cov->n_fc);
      int64_t off = 0, n_lt = 0, n_gt = 0, koff = 0;
      // stored coupling matrices, one per geometry of an ordered pair (target
      // c, partner t): K(xi_t, xi_c) row-major with the partner's nodes as
      // rows; far list entries of the same geometry share it
      double qscale;
      {
        std::vector<const double *> cs, hs;
        for (const FarCluster &c : fcs) {
          cs.push_back(c.ctr);
          hs.push_back(c.hw);
        }
        qscale = coupling_quantum(d, cs, hs);
      }
      std::map<std::vector<int64_t>, int64_t> kshape;
      std::vector<PairItem> uprs;
      std::vector<int64_t> fko(fcol.size());
      for (int c = 0; c < cov->n_fc; ++c)
        for (int e = fp[c]; e < fp[c + 1]; ++e) {
          const FarCluster &tg = fcs[c], &pt = fcs[fcol[e]];
          std::vector<int64_t> key = coupling_key(d, pt.p, tg.p, pt.ctr, pt.hw, tg.ctr, tg.hw,
                                                  qscale);
          auto it = kshape.find(key);
          if (it != kshape.end()) {
            fko[e] = it->second;
          } else {
            PairItem q{};
            q.s = fcol[e];
            q.t = c;
            q.koff = koff;
            uprs.push_back(q);
            kshape.emplace(std::move(key), koff);
            fko[e] = koff;
            koff += (int64_t)pt.pd * tg.pd;
          }
        }
      int64_t n_kpair = 0;
      for (auto &pr : fpairs) {
        if (pr.first < pr.second) {
          ++n_lt;
          const int pds = fcs[pr.first].pd, pdt = fcs[pr.second].pd;
          const int nrb = (pds + kRowBlk - 1) / kRowBlk, ncb = (pdt + 63) / 64;
          PairItem q{};
          q.s = pr.first;
          q.t = pr.second;
          q.off = off;
          for (int cb = 0; cb < ncb; ++cb) cpl[pr.first].push_back(off + (int64_t)cb * pds);
          for (int rb = 0; rb < nrb; ++rb)
            cpl[pr.second].push_back(off + (int64_t)ncb * pds + (int64_t)rb * pdt);
          for (int rb = 0; rb < nrb; ++rb)
            for (int cb = 0; cb < ncb; ++cb)
              cis.push_back(CoupleItem{(int32_t)prs.size(), (int16_t)rb, (int16_t)cb});
          off += (int64_t)ncb * pds + (int64_t)nrb * pdt;
          n_kpair += (int64_t)pds * pdt;
          prs.push_back(q);
        } else {
          ++n_gt;
        }
      }
      if (n_lt != n_gt) throw Error{FKF_E_ARG, "fkf_cov_build: admissible pairs are not symmetric"};
      cov->n_kst = koff;
      cov->n_kpair = n_kpair;
      cov->n_pairs = (int64_t)prs.size();
      cov->n_part_pair = off;
      cov->n_citems = (int64_t)cis.size();
      cov->citems.upload(cis, st);
      cov->pairs.upload(prs, st);
      cov->n_upairs = (int64_t)uprs.size();
      cov->upairs.upload(uprs, st);
      cov->far_koff.upload(fko, st);
      {
        // groups of targets with the same sequence of stored matrices (far
        // list sorted by matrix, ties by partner): key = pd, then the
        // (matrix, partner pd) pairs
        std::map<std::vector<int64_t>, int> gid;
        std::vector<std::vector<int>> members;
        std::vector<std::vector<std::pair<int64_t, int>>> gseq;
        std::vector<std::vector<int32_t>> tx(cov->n_fc);   // sorted partner coef offsets
        bool fits = cov->n_coef < (int64_t)INT32_MAX;
        for (int c = 0; c < cov->n_fc && fits; ++c) {
          std::vector<std::pair<int64_t, int>> ent;   // (matrix, partner)
          for (int e = fp[c]; e < fp[c + 1]; ++e) ent.emplace_back(fko[e], fcol[e]);
          std::sort(ent.begin(), ent.end());
          std::vector<int64_t> key{fcs[c].pd};
          for (auto &q : ent) {
            key.push_back(q.first);
            key.push_back(fcs[q.second].pd);
            tx[c].push_back((int32_t)fcs[q.second].coef_off);
          }
          auto it = gid.find(key);
          if (it == gid.end()) {
            it = gid.emplace(std::move(key), (int)members.size()).first;
            members.emplace_back();
            std::vector<std::pair<int64_t, int>> sq;
            for (auto &q : ent) sq.emplace_back(q.first, fcs[q.second].pd);
            gseq.push_back(std::move(sq));
          }
          members[it->second].push_back(c);
        }
        // worth it when the groups are large (a regular grid) and the
        // couplings are FP64 (measured on the 256 x 256 grid: 50 us against
        // 70 us per target in FP64, but 51 us against 36 us in FP32, whose
        // per-target reads of the stored matrices are half as many bytes);
        // irregular points keep the per-target kernel
        if (!cov->mixed && fits && !members.empty() &&
            cov->n_fc >= 4 * (int64_t)members.size()) {
          std::vector<int64_t> gk;
          std::vector<int32_t> gpd, tcoef, xoff;
          std::vector<std::pair<int64_t, GroupItem>> items;
          for (size_t g = 0; g < members.size(); ++g) {
            const int seq = (int)gk.size(), len = (int)gseq[g].size();
            int64_t work = 0;
            for (auto &q : gseq[g]) {
              gk.push_back(q.first);
              gpd.push_back(q.second);
              work += q.second;
            }
            const int pd = fcs[members[g][0]].pd;
            for (size_t i0 = 0; i0 < members[g].size(); i0 += kGrpSlots) {
              const int slot0 = (int)tcoef.size(), xbase = (int)xoff.size();
              const int ns = (int)std::min<size_t>(kGrpSlots, members[g].size() - i0);
              for (int i = 0; i < ns; ++i) {
                const int c = members[g][i0 + i];
                tcoef.push_back((int32_t)fcs[c].coef_off);
                xoff.insert(xoff.end(), tx[c].begin(), tx[c].end());
              }
              for (int rb = 0; rb * 64 < pd; ++rb) {
                GroupItem gi{seq, len, pd, rb, slot0, ns, xbase, 0};
                items.emplace_back(-work * std::min(64, pd - 64 * rb), gi);
              }
            }
          }
          std::stable_sort(items.begin(), items.end(),
                           [](const auto &a, const auto &b) { return a.first < b.first; });
          std::vector<GroupItem> gi;
          for (auto &q : items) gi.push_back(q.second);
          cov->n_grp_items = (int64_t)gi.size();
          cov->n_grp_groups = (int64_t)members.size();
          cov->grp_items.upload(gi, st);
          cov->grp_koff.upload(gk, st);
          cov->grp_pdt.upload(gpd, st);
          cov->grp_tcoef.upload(tcoef, st);
          cov->grp_xoff.upload(xoff.empty() ? std::vector<int32_t>(1, 0) : xoff, st);
          cov->grouped = true;
          FKF_CHECK_HIP(hipStreamSynchronize(st));   // host temporaries
        }
      }
      FKF_CHECK_HIP(hipStreamSynchronize(st));   // prs, uprs, fko are host temporaries
      std::vector<int32_t> cptr(1, 0);
      std::vector<int64_t> coff;
      for (auto &v : cpl) {
        coff.insert(coff.end(), v.begin(), v.end());
        cptr.push_back((int32_t)coff.size());
      }
      cov->cp_ptr.upload(cptr, st);
      cov->cp_off.upload(coff, st);
    }
    std::vector<double> ch((kMaxCheb + 1) * 2 * kMaxCheb, 0.0);
    for (int p = 1; p <= kMaxCheb; ++p) cheb_nodes(p, &ch[p * 2 * kMaxCheb], &ch[p * 2 * kMaxCheb + kMaxCheb]);
    cov->cheb.upload(ch, st);
    // Lagrange table of the several-column upward pass (needs the node table)
    if (cov->n_up_items_m > 0) {
      const unsigned gy = (unsigned)((kUpChunkM * d + 255) / 256);
      if (d == 2)
        hipLaunchKernelGGL(k_lagrange_table<2>, dim3((unsigned)cov->n_up_items_m, gy), dim3(256), 0,
                           st, cov->up_items_m.p, cov->fc.p, cov->pts.p, n, cov->cheb.p,
                           cov->lag.p);
      else
        hipLaunchKernelGGL(k_lagrange_table<3>, dim3((unsigned)cov->n_up_items_m, gy), dim3(256), 0,
                           st, cov->up_items_m.p, cov->fc.p, cov->pts.p, n, cov->cheb.p,
                           cov->lag.p);
      FKF_CHECK_HIP(hipGetLastError());
    }
    const int64_t kbytes = cov->n_kst * (int64_t)(cov->mixed ? sizeof(float) : sizeof(double));
    if (cov->n_pairs > 0 && kbytes <= kMaxCouplingBytes && hp->far_eval == 0) {
      void *dst;
      if (cov->mixed) {
        cov->kst32.alloc((size_t)cov->n_kst);
        dst = cov->kst32.p;
      } else {
        cov->kst.alloc((size_t)cov->n_kst);
        dst = cov->kst.p;
      }
      auto store = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((unsigned)cov->n_upairs), dim3(256), 0, st, cov->upairs.p,
                           cov->fc.p, cov->cheb.p, cov->kind, 1.0 / cov->ell, cov->amp, dst);
      };
      if (d == 3)
        cov->mixed ? store(k_couple_store<3, true>) : store(k_couple_store<3, false>);
      else
        cov->mixed ? store(k_couple_store<2, true>) : store(k_couple_store<2, false>);
      cov->stored = true;
    }
    // second stream and fork/join events of the products (the near field
    // runs beside the far-field chain)
    FKF_CHECK_HIP(hipStreamCreateWithFlags(&cov->side, hipStreamNonBlocking));
    FKF_CHECK_HIP(hipEventCreateWithFlags(&cov->ev_fork, hipEventDisableTiming));
    FKF_CHECK_HIP(hipEventCreateWithFlags(&cov->ev_join, hipEventDisableTiming));
    FKF_CHECK_HIP(hipStreamSynchronize(st));
    *out = cov.release();
  });
}

namespace {

// One column: near field (HBM-bound) on a forked stream, far field (ALU-bound)
// on the caller's stream, joined before the final pass.
// Second stream (default priority) and fork/join events of a covariance
// operator, created by fkf_cov_build.
static void ensure_side_stream(fkf_cov *cov) {
  if (!cov->side) throw Error{FKF_E_ORDER, "covariance operator has no side stream"};
}

void apply_one(fkf_cov *cov, const ApplyWs &ws, double *Y, hipStream_t st) {
  const int64_t n = cov->n;
  ensure_side_stream(cov);
  FKF_CHECK_HIP(hipEventRecord(cov->ev_fork, st));
  FKF_CHECK_HIP(hipStreamWaitEvent(cov->side, cov->ev_fork, 0));
  {
    FKF_TRACE("hmat_near_1rhs", cov->side);
    if (cov->n_blk && cov->mixed)
      hipLaunchKernelGGL(k_near_sym1_32, dim3((unsigned)((cov->n_blk + 3) / 4)), dim3(256), 0,
                         cov->side, cov->blk32.p, cov->blk_s.p, cov->blk_t.p, cov->leaf_off.p,
                         ws.xt, cov->n_blk, ws.part);
    else if (cov->n_blk)
      hipLaunchKernelGGL(k_near_sym1, dim3((unsigned)((cov->n_blk + 3) / 4)), dim3(256), 0,
                         cov->side, cov->blk.p, cov->blk_s.p, cov->blk_t.p, cov->leaf_off.p,
                         ws.xt, cov->n_blk, ws.part);
  }
  FKF_CHECK_HIP(hipEventRecord(cov->ev_join, cov->side));
  const bool d3 = cov->d == 3;
  if (cov->n_fc > 0) {
    {
      FKF_TRACE("hmat_far_up_1rhs", st);
      if (d3)
        hipLaunchKernelGGL(k_up1<3>, dim3((unsigned)cov->n_up_items), dim3(64), 0, st,
                           cov->up_items.p, cov->fc.p, cov->pts.p, n, cov->cheb.p, ws.xt,
                           ws.part_up);
      else
        hipLaunchKernelGGL(k_up1_mfma2, dim3((unsigned)cov->n_up_items), dim3(64), 0, st,
                           cov->up_items.p, cov->fc.p, cov->pts.p, n, cov->cheb.p, ws.xt,
                           ws.part_up);
      hipLaunchKernelGGL(k_up_reduce, dim3((cov->n_fc + 3) / 4), dim3(256), 0, st, cov->fc.p,
                         cov->n_fc, cov->up_ptr.p,
                         cov->up_items.p, ws.part_up, ws.xhat);
    }
    {
      FKF_TRACE("hmat_far_couple_1rhs", st);
      auto launch = [&](auto kern) {
        if (cov->n_citems > 0)
          hipLaunchKernelGGL(kern, dim3((unsigned)((cov->n_citems + 3) / 4)), dim3(256), 0, st,
                           cov->citems.p, cov->n_citems, cov->pairs.p, cov->fc.p, cov->cheb.p,
                           cov->kind, 1.0 / cov->ell, cov->amp, ws.xhat,
                           ws.part_pair);
      };
      if (cov->stored && cov->grouped) {   // FP64 couplings only
        hipLaunchKernelGGL(k_couple_grp1<double>, dim3((unsigned)cov->n_grp_items), dim3(512), 0,
                           st, cov->grp_items.p, cov->grp_koff.p, cov->grp_pdt.p, cov->grp_tcoef.p,
                           cov->grp_xoff.p, cov->kst.p, ws.xhat, ws.yhat);
      } else if (cov->stored) {
        const dim3 g((unsigned)cov->n_fc, (unsigned)((cov->max_pd + 63) / 64));
        if (cov->mixed)
          hipLaunchKernelGGL(k_couple_rows1<float>, g, dim3(256), 0, st, cov->fc.p,
                             cov->far_ptr.p, cov->far_col.p, cov->far_koff.p, cov->kst32.p,
                             ws.xhat, ws.yhat);
        else
          hipLaunchKernelGGL(k_couple_rows1<double>, g, dim3(256), 0, st, cov->fc.p,
                             cov->far_ptr.p, cov->far_col.p, cov->far_koff.p, cov->kst.p,
                             ws.xhat, ws.yhat);
      } else {
        const int sel = (d3 ? 2 : 0) + (cov->mixed ? 1 : 0);
        switch (sel) {
          case 0: launch(k_couple_blk<2, false>); break;
          case 1: launch(k_couple_blk<2, true>); break;
          case 2: launch(k_couple_blk<3, false>); break;
          default: launch(k_couple_blk<3, true>); break;
        }
        hipLaunchKernelGGL(k_couple_reduce, dim3((cov->n_fc + 3) / 4), dim3(256), 0, st,
                           cov->fc.p, cov->n_fc, cov->cp_ptr.p, cov->cp_off.p, ws.part_pair,
                           ws.yhat);
      }
    }
  }
  FKF_CHECK_HIP(hipStreamWaitEvent(st, cov->ev_join, 0));
  {
    FKF_TRACE("hmat_final_1rhs", st);
    if (d3)
      hipLaunchKernelGGL(k_final1<3>, dim3(cov->n_leaves), dim3(256), 0, st, cov->leaf_off.p,
                         cov->pts.p, n, cov->cheb.p, cov->fc.p, cov->anc_ptr.p, cov->anc_idx.p,
                         ws.yhat, ws.part, cov->part_ptr.p, cov->part_idx.p, cov->perm.p,
                         Y);
    else
      hipLaunchKernelGGL(k_final1_mfma2, dim3(cov->n_leaves), dim3(256), 0, st, cov->leaf_off.p,
                         cov->pts.p, n, cov->cheb.p, cov->fc.p, cov->anc_ptr.p, cov->anc_idx.p,
                         ws.yhat, ws.part, cov->part_ptr.p, cov->part_idx.p, cov->perm.p,
                         Y);
  }
}

// Near field of the several-column product (written to Y in caller order).
template <bool F32>
void near_multi(fkf_cov *cov, const ApplyWs &ws, int nrhs, double *Y, int64_t ldy, hipStream_t s) {
  typedef typename std::conditional<F32, float, double>::type TT;
  const TT *frag = F32 ? (const TT *)cov->frag32.p : (const TT *)cov->frag.p;
  hipLaunchKernelGGL(k_near_mfma<TT>, dim3(cov->n_leaves, (unsigned)((nrhs + 127) / 128)),
                     dim3(512), 0, s, frag, cov->near_ptr.p, cov->near_idx.p, cov->blk_s.p,
                     cov->blk_t.p, cov->leaf_off.p, cov->n, ws.xt, cov->perm.p, nrhs, Y, ldy);
}

// ------------------------------------------- sparse right-hand sides ---
// The columns of the several-column product may be the rows of a sparse
// matrix (the transposed measurement operator: a ray crosses O(sqrt n)
// cells).  The moments U_c^T X_c of a far cluster c then reduce to sums over
// the nonzeros inside c, which replaces the upward pass's dense products
// (the paper applies the covariance to the dense columns; the sums are the
// same up to rounding order).

// Rows longer than this are not taken by the sparse moments (LDS sort size).
constexpr int kSpRowMax = 2048;

// One workgroup per row j = j0 + blockIdx.x of the sparse matrix: its
// entries moved to tree order (position iperm[col]) and sorted ascending
// (bitonic sort in LDS of the key (position, entry), so equal positions keep
// their order), written to tix / val at the row's offset; and for every leaf
// boundary s = 0 .. n_leaves the number of the row's entries in leaves
// before s, cnt[blockIdx.x (n_leaves + 1) + s] (rows of the current column
// block).  The host guarantees len <= kSpRowMax.
__global__ void __launch_bounds__(256) k_sparse_rows(
    const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const int32_t *__restrict__ iperm,
    const int64_t *__restrict__ leaf_off, int n_leaves, int j0, const int32_t *__restrict__ order,
    int32_t *__restrict__ tix, double *__restrict__ tval, int32_t *__restrict__ cnt) {
  __shared__ int64_t key[kSpRowMax];
  const int j = order ? order[j0 + blockIdx.x] : j0 + blockIdx.x, tid = threadIdx.x;
  const int64_t e0 = rowptr[j];
  const int len = (int)(rowptr[j + 1] - e0);
  int m = 1;
  while (m < len) m <<= 1;
  for (int e = tid; e < m; e += 256)
    key[e] = e < len ? ((int64_t)iperm[col[e0 + e]] << 32) | e : INT64_MAX;
  __syncthreads();
  for (int k = 2; k <= m; k <<= 1)
    for (int h = k >> 1; h > 0; h >>= 1) {
      for (int i = tid; i < m; i += 256) {
        const int x = i ^ h;
        if (x > i) {
          const int64_t a = key[i], b = key[x];
          if ((a > b) == ((i & k) == 0)) {
            key[i] = b;
            key[x] = a;
          }
        }
      }
      __syncthreads();
    }
  const int64_t o = e0 - rowptr[0];
  for (int e = tid; e < len; e += 256) {
    const int64_t kv = key[e];
    tix[o + e] = (int32_t)(kv >> 32);
    tval[o + e] = val[e0 + (kv & 0xffffffff)];
  }
  for (int q = tid; q <= n_leaves; q += 256) {
    const int64_t b = leaf_off[q];
    int lo = 0, hi = len;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((key[mid] >> 32) < b) lo = mid + 1;
      else hi = mid;
    }
    cnt[(int64_t)blockIdx.x * (n_leaves + 1) + q] = lo;
  }
}

// Nonzero flags of the sparse moments, one thread per (far cluster c, block
// b of 16 rows of the current column block): nzb[c ncb16 + b] = 1 when one of
// the block's rows 16 b .. 16 b + 15 (< nrhs; counts by row of the column
// block) has an entry inside c.
__global__ void __launch_bounds__(256) k_sparse_nzb(const int32_t *__restrict__ fc_leaf,
                                                    int n_fc, const int32_t *__restrict__ cnt,
                                                    int n_leaves, int nrhs,
                                                    int32_t *__restrict__ nzb) {
  const int ncb16 = (nrhs + 15) >> 4;
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)n_fc * ncb16) return;
  const int c = (int)(g / ncb16), b = (int)(g % ncb16);
  const int L0 = fc_leaf[2 * c], L1 = fc_leaf[2 * c + 1];
  int any = 0;
  for (int q = 0; q < 16; ++q) {
    const int jj = 16 * b + q;
    if (jj < nrhs) {
      const int32_t *cj = cnt + (int64_t)jj * (n_leaves + 1);
      any |= cj[L1] > cj[L0];
    }
  }
  nzb[g] = any;
}

// Nonzero 16-column blocks of each far cluster's Yhat: block b of cluster s
// is nonzero when block b of some partner's moments is (nzb of the partners).
__global__ void __launch_bounds__(256) k_sparse_ynz(const int32_t *__restrict__ far_ptr,
                                                    const int32_t *__restrict__ far_col,
                                                    int n_fc, int ncb16,
                                                    const int32_t *__restrict__ nzb,
                                                    int32_t *__restrict__ ynz) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)n_fc * ncb16) return;
  const int c = (int)(g / ncb16), b = (int)(g % ncb16);
  int any = 0;
  for (int e = far_ptr[c]; e < far_ptr[c + 1] && !any; ++e)
    any = nzb[(int64_t)far_col[e] * ncb16 + b];
  ynz[g] = any;
}

// Partners of far cluster s whose moments are not all zero in the 256-column
// block cb (some of its 16-column blocks 16 cb .. 16 cb + 15 marked in nzb),
// in far-list order: plist[far_ptr[s] ncbw + cb deg(s) + i], i < pcnt[s ncbw
// + cb] (deg(s) = far_ptr[s + 1] - far_ptr[s]).  One wavefront per (s, cb),
// lanes over up to 64 partners at a time.
__global__ void __launch_bounds__(256) k_sparse_plist(const int32_t *__restrict__ far_ptr,
                                                      const int32_t *__restrict__ far_col,
                                                      int n_fc, int ncb16, int ncbw,
                                                      const int32_t *__restrict__ nzb,
                                                      int32_t *__restrict__ plist,
                                                      int32_t *__restrict__ pcnt) {
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (g >= (int64_t)n_fc * ncbw) return;
  const int l = threadIdx.x & 63;
  const int s = (int)(g / ncbw), cb = (int)(g % ncbw);
  const int e0 = far_ptr[s], e1 = far_ptr[s + 1];
  const int b0 = 16 * cb, b1 = min(ncb16, b0 + 16);
  int32_t *out = plist + (int64_t)e0 * ncbw + (int64_t)cb * (e1 - e0);
  int n = 0;
  for (int eb = e0; eb < e1; eb += 64) {
    const int e = eb + l;
    int any = 0;
    if (e < e1) {
      const int32_t *f = nzb + (int64_t)far_col[e] * ncb16;
      for (int b = b0; b < b1; ++b) any |= f[b];
    }
    const uint64_t m = __ballot(any != 0);
    if (any) out[n + __popcll(m & ((1ull << l) - 1))] = e;
    n += __popcll(m);
  }
  if (l == 0) pcnt[g] = n;
}

// Moments of far cluster c = blockIdx.x: xhat[c.coef_off nrhs + a + pd (j -
// j0)] = sum over row j's entries (i, v) inside c of v * prod_k
// l_{a_k}(z_k(x_i)), in the sorted order; the entries inside c are those
// between the counts at the cluster's first and end leaf.  Rows without
// entries in c give zeros; 16-column blocks marked zero in nzb are not
// written (the couplings never read them).  Lanes run over the
// coefficients a, four entries' loads in flight.  Clusters of more than
// kUpBlockPts points: one wavefront per row (rows j0 + 4 blockIdx.y + w);
// smaller ones, whose rows hold few entries: one wavefront per 16-row block
// (block 4 blockIdx.y + w), the rows' counts read at once (one row per lane)
// and the rows taken in turn, zero rows written without further loads.
constexpr int64_t kUpBlockPts = 512;

template <int D>
__device__ __forceinline__ void up_sparse_row(const FarCluster &c, const double *__restrict__ lag,
                                              const int32_t *__restrict__ tix,
                                              const double *__restrict__ tval, int64_t lo,
                                              int64_t hi, double *__restrict__ o, int l) {
  constexpr int PM = PMax<D>::v;
  for (int a0 = 0; a0 < c.pd; a0 += 64) {
    const int a = a0 + l;
    int dig[D];
    {
      int r = a < c.pd ? a : 0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        dig[k] = r % c.p;
        r /= c.p;
      }
    }
    // four entries' loads in flight at a time; the sum keeps the sorted order
    double acc = 0.0;
    int64_t e = lo;
    for (; e + 4 <= hi; e += 4) {
      double v[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double *L = lag + c.lag_off + (int64_t)(tix[e + u] - c.begin) * D * PM;
        v[u] = tval[e + u];
        b[u] = L[dig[0]];
#pragma unroll
        for (int k = 1; k < D; ++k) b[u] *= L[k * PM + dig[k]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = fma(v[u], b[u], acc);
    }
    for (; e < hi; ++e) {
      const double *L = lag + c.lag_off + (int64_t)(tix[e] - c.begin) * D * PM;
      double b = L[dig[0]];
#pragma unroll
      for (int k = 1; k < D; ++k) b *= L[k * PM + dig[k]];
      acc = fma(tval[e], b, acc);
    }
    if (a < c.pd) o[a] = acc;
  }
}

template <int D>
__global__ void __launch_bounds__(256) k_up_sparse(
    const FarCluster *__restrict__ fc, const int32_t *__restrict__ fc_leaf,
    const double *__restrict__ lag, const int64_t *__restrict__ rowptr, int j0,
    const int32_t *__restrict__ order, int nrhs, const int32_t *__restrict__ tix,
    const double *__restrict__ tval, const int32_t *__restrict__ cnt, int n_leaves,
    const int32_t *__restrict__ nzb, double *__restrict__ xhat) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int ncb16 = (nrhs + 15) >> 4;
  const FarCluster c = fc[blockIdx.x];
  const int L0 = fc_leaf[2 * blockIdx.x], L1 = fc_leaf[2 * blockIdx.x + 1];
  double *oc = xhat + c.coef_off * nrhs;
  if (c.end - c.begin > kUpBlockPts) {
    const int jj = blockIdx.y * 4 + w;
    if (jj >= nrhs) return;
    // a column whose 16-column block of this cluster is zero is never read
    // (the couplings skip such blocks): nothing to write
    if (!nzb[(int64_t)blockIdx.x * ncb16 + (jj >> 4)]) return;
    const int j = order ? order[j0 + jj] : j0 + jj;
    const int32_t *cj = cnt + (int64_t)jj * (n_leaves + 1);
    const int64_t base = rowptr[j] - rowptr[0];
    up_sparse_row<D>(c, lag, tix, tval, base + cj[L0], base + cj[L1], oc + (int64_t)c.pd * jj,
                     l);
    return;
  }
  const int b = blockIdx.y * 4 + w;   // 16-row block
  if (b >= ncb16) return;
  if (!nzb[(int64_t)blockIdx.x * ncb16 + b]) return;
  const int jb = 16 * b, nq = min(16, nrhs - jb);
  // lane q < nq: the entries of row jb + q inside c
  int64_t lo_l = 0, hi_l = 0;
  if (l < nq) {
    const int jj = jb + l;
    const int j = order ? order[j0 + jj] : j0 + jj;
    const int32_t *cj = cnt + (int64_t)jj * (n_leaves + 1);
    const int64_t base = rowptr[j] - rowptr[0];
    lo_l = base + cj[L0];
    hi_l = base + cj[L1];
  }
  for (int q = 0; q < nq; ++q) {
    const int64_t lo = ((int64_t)__builtin_amdgcn_readlane((int)(lo_l >> 32), q) << 32) |
                       (uint32_t)__builtin_amdgcn_readlane((int)lo_l, q);
    const int64_t hi = ((int64_t)__builtin_amdgcn_readlane((int)(hi_l >> 32), q) << 32) |
                       (uint32_t)__builtin_amdgcn_readlane((int)hi_l, q);
    double *o = oc + (int64_t)c.pd * (jb + q);
    if (lo == hi) {
      for (int a = l; a < c.pd; a += 64) o[a] = 0.0;
    } else {
      up_sparse_row<D>(c, lag, tix, tval, lo, hi, o, l);
    }
  }
}

// Near field of the several-column product for sparse columns:
// Y[perm[s0 + i], j - j0] = sum over the near pairs e = (s, t) of target leaf
// s, in list order, of sum over row j's entries (p, v) inside leaf t, in
// sorted order, of A_st[i, p - t0] v, with the entries of A_st read from the
// repacked tiles (the values the dense near field multiplies; entry (i, k) of
// tile e at e 4096 + (i / 16) 1024 + (k / 4) 64 + (k % 4) 16 + i % 16).  One
// workgroup per (target leaf s = blockIdx.x, 4 rows), one wavefront per row
// j, lanes over the leaf's points.  Rows without entries near s give zeros.
// The counts of up to 64 near pairs are read at once (one pair per lane) and
// only the pairs that hold entries of the row are visited; a pair's entries
// are read 64 at a time and taken in turn across lanes, four tile entries in
// flight.
template <typename TT>
__global__ void __launch_bounds__(256) k_near_sparse(
    const TT *__restrict__ frag, const int32_t *__restrict__ near_ptr,
    const int32_t *__restrict__ near_src, const int64_t *__restrict__ leaf_off,
    const int64_t *__restrict__ rowptr, int j0, const int32_t *__restrict__ order, int nrhs,
    const int32_t *__restrict__ tix, const double *__restrict__ tval,
    const int32_t *__restrict__ cnt, int n_leaves, const int64_t *__restrict__ perm,
    double *__restrict__ Y, int64_t ldy) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int jj = blockIdx.y * 4 + w;
  if (jj >= nrhs) return;
  const int s = blockIdx.x, j = order ? order[j0 + jj] : j0 + jj;
  const int e0 = near_ptr[s], e1 = near_ptr[s + 1];
  const int64_t s0 = leaf_off[s], ms = leaf_off[s + 1] - s0;
  const int32_t *cj = cnt + (int64_t)jj * (n_leaves + 1);
  const int64_t base = rowptr[j] - rowptr[0];
  const int ir = l < ms ? l : 0;
  const int64_t rowoff = (ir >> 4) * 1024 + (ir & 15);
  double acc = 0.0;
  for (int eb = e0; eb < e1; eb += 64) {
    int t = 0, clo = 0, chi = 0;
    if (eb + l < e1) {
      t = near_src[eb + l];
      clo = cj[t];
      chi = cj[t + 1];
    }
    uint64_t m = __ballot(chi > clo);
    while (m) {
      const int q = __builtin_ctzll(m);
      m &= m - 1;
      const int64_t lo = base + __builtin_amdgcn_readlane(clo, q);
      const int64_t hi = base + __builtin_amdgcn_readlane(chi, q);
      const int64_t t0 = leaf_off[__builtin_amdgcn_readlane(t, q)];
      const TT *A = frag + (int64_t)(eb + q) * 4096 + rowoff;
      for (int64_t h0 = lo; h0 < hi; h0 += 64) {
        const int n = (int)min((int64_t)64, hi - h0);
        int k = 0;
        double v = 0.0;
        if (l < n) {
          k = (int)(tix[h0 + l] - t0);
          v = tval[h0 + l];
        }
        const int64_t vb = __double_as_longlong(v);
        const int vlo = (int)vb, vhi = (int)(vb >> 32);
        int u = 0;
        for (; u + 4 <= n; u += 4) {
          double a[4], vv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int kr = __builtin_amdgcn_readlane(k, u + r);
            a[r] = (double)A[(kr >> 2) * 64 + (kr & 3) * 16];
            vv[r] = __longlong_as_double(
                ((int64_t)__builtin_amdgcn_readlane(vhi, u + r) << 32) |
                (uint32_t)__builtin_amdgcn_readlane(vlo, u + r));
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) acc = fma(a[r], vv[r], acc);
        }
        for (; u < n; ++u) {
          const int kr = __builtin_amdgcn_readlane(k, u);
          const double vu = __longlong_as_double(
              ((int64_t)__builtin_amdgcn_readlane(vhi, u) << 32) |
              (uint32_t)__builtin_amdgcn_readlane(vlo, u));
          acc = fma((double)A[(kr >> 2) * 64 + (kr & 3) * 16], vu, acc);
        }
      }
    }
  }
  if (l < ms) Y[perm[s0 + l] + ldy * (int64_t)j] = acc;   // column of row j of H
}

// Columns of a several-column product given as sparse rows: row pointers
// (device) and the first row j0 of the current column block.
struct SparseRhs {
  const int64_t *rowptr;
  int j0;
  const int32_t *order;   // column c of the product is row order[c] of H (null: row c)
};

// Several columns on the FP64 matrix cores: the near field on a forked
// stream, concurrently with the far-field chain (upward chunks + reduction,
// couplings per cluster row block); the downward pass then adds to Y.  With
// sparse rows (sp), column c of the block is row r = sp->order[sp->j0 + c]
// (or sp->j0 + c) of H and lands in column r of Y (Y not offset by the block).
template <int D, bool F32>
void apply_multi_t(fkf_cov *cov, const ApplyWs &ws, int nrhs, double *Y, int64_t ldy,
                   hipStream_t st, const SparseRhs *sp) {
  const int64_t n = cov->n;
  if (cov->n_fc > 0) {
    // near field on the side stream, concurrent with the far-field chain;
    // the downward pass then adds to its result.  The sparse near field is
    // forked after the sparse upward pass: both are latency-bound and gain
    // nothing side by side, while the couplings leave it room
    ensure_side_stream(cov);
    auto fork_near = [&] {
      FKF_CHECK_HIP(hipEventRecord(cov->ev_fork, st));
      FKF_CHECK_HIP(hipStreamWaitEvent(cov->side, cov->ev_fork, 0));
      if (sp) {
        FKF_TRACE("hmat_near_sparse", cov->side);
        typedef typename std::conditional<F32, float, double>::type TT;
        const TT *frag = F32 ? (const TT *)cov->frag32.p : (const TT *)cov->frag.p;
        hipLaunchKernelGGL(k_near_sparse<TT>, dim3(cov->n_leaves, (unsigned)((nrhs + 3) / 4)),
                           dim3(256), 0, cov->side, frag, cov->near_ptr.p, cov->near_src.p,
                           cov->leaf_off.p, sp->rowptr, sp->j0, sp->order, nrhs,
                           cov->sp_tix.p, cov->sp_val.p, cov->sp_cnt.p, cov->n_leaves,
                           cov->perm.p, Y, ldy);
      } else {
        FKF_TRACE("hmat_near_multi", cov->side);
        near_multi<F32>(cov, ws, nrhs, Y, ldy, cov->side);
      }
      FKF_CHECK_HIP(hipEventRecord(cov->ev_join, cov->side));
    };
    if (!sp) fork_near();
    if (sp) {
      FKF_TRACE("hmat_far_up_sparse", st);
      // zero 16-column blocks of every far cluster's moments (from the
      // per-leaf counts of the rows), then the moments of the others
      const int64_t nf = (int64_t)cov->n_fc * ((nrhs + 15) / 16);
      cov->sp_nzb.reserve((size_t)nf);
      hipLaunchKernelGGL(k_sparse_nzb, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st,
                         cov->fc_leaf.p, cov->n_fc, cov->sp_cnt.p, cov->n_leaves, nrhs,
                         cov->sp_nzb.p);
      hipLaunchKernelGGL((k_up_sparse<D>), dim3((unsigned)cov->n_fc, (unsigned)((nrhs + 3) / 4)),
                         dim3(256), 0, st, cov->fc.p, cov->fc_leaf.p, cov->lag.p, sp->rowptr,
                         sp->j0, sp->order, nrhs, cov->sp_tix.p, cov->sp_val.p, cov->sp_cnt.p,
                         cov->n_leaves, cov->sp_nzb.p, ws.xhat);
      cov->sp_ynz.reserve((size_t)nf);
      hipLaunchKernelGGL(k_sparse_ynz, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st,
                         cov->far_ptr.p, cov->far_col.p, cov->n_fc, (nrhs + 15) / 16,
                         cov->sp_nzb.p, cov->sp_ynz.p);
      const int ncbw = (nrhs + 255) / 256;   // column blocks of the couplings' workgroups
      const int64_t nl = (int64_t)cov->n_fc * ncbw;
      cov->sp_plist.reserve(std::max<size_t>(cov->far_col.n * (size_t)ncbw, 1));
      cov->sp_pcnt.reserve((size_t)std::max<int64_t>(nl, 1));
      hipLaunchKernelGGL(k_sparse_plist, dim3((unsigned)((nl + 3) / 4)), dim3(256), 0, st,
                         cov->far_ptr.p, cov->far_col.p, cov->n_fc, (nrhs + 15) / 16, ncbw,
                         cov->sp_nzb.p, cov->sp_plist.p, cov->sp_pcnt.p);
      fork_near();
    } else {
      FKF_TRACE("hmat_far_up_multi", st);
      hipLaunchKernelGGL((k_up_mfma2<D>),
                         dim3((unsigned)cov->n_up_blocks_m, (unsigned)((nrhs + 511) / 512)),
                         dim3(512), 0, st, cov->up_blocks_m.p, cov->up_items_m.p, cov->fc.p,
                         cov->lag.p, n, ws.xt, nrhs, ws.part_up_m);
      hipLaunchKernelGGL(k_up_reduce_m, dim3(cov->n_fc, 8), dim3(256), 0, st, cov->fc.p,
                         cov->up_ptr_m.p, cov->up_items_m.p, nrhs, ws.part_up_m, ws.xhat);
    }
    {
      FKF_TRACE("hmat_far_couple_multi", st);
      // clusters without partners get zero coefficients
      if (!cov->cm_all) {
        const int64_t len = cov->n_coef * nrhs;
        hipLaunchKernelGGL(k_zero, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st,
                           ws.yhat, len);
      }
      const int32_t *nzb = sp ? cov->sp_nzb.p : nullptr;   // formed before the upward pass
      const int32_t *plist = sp ? cov->sp_plist.p : nullptr, *pcnt = sp ? cov->sp_pcnt.p : nullptr;
      if (cov->n_cm_items > 0) {
        // couplings read from the stored matrices where they are kept, else
        // evaluated into LDS chunk by chunk
        const dim3 grid((unsigned)cov->n_cm_items, (unsigned)((nrhs + 255) / 256));
        const void *kst = F32 ? (const void *)cov->kst32.p : (const void *)cov->kst.p;
        if (cov->stored)
          hipLaunchKernelGGL((k_couple_mfma2<D, F32, true>), grid, dim3(512), 0, st,
                             cov->cm_items.p, cov->fc.p, cov->far_ptr.p, cov->far_col.p,
                             cov->cheb.p, cov->kind, 1.0 / cov->ell, cov->amp, cov->far_koff.p,
                             kst, ws.xhat, nrhs, ws.yhat, nzb, plist, pcnt);
        else
          hipLaunchKernelGGL((k_couple_mfma2<D, F32, false>), grid, dim3(512), 0, st,
                             cov->cm_items.p, cov->fc.p, cov->far_ptr.p, cov->far_col.p,
                             cov->cheb.p, cov->kind, 1.0 / cov->ell, cov->amp, nullptr,
                             nullptr, ws.xhat, nrhs, ws.yhat, nzb, plist, pcnt);
      }
    }
  }
  if (cov->n_fc == 0) {
    FKF_TRACE("hmat_near_multi", st);
    near_multi<F32>(cov, ws, nrhs, Y, ldy, st);
    return;
  }
  FKF_TRACE("hmat_down_multi", st);
  FKF_CHECK_HIP(hipStreamWaitEvent(st, cov->ev_join, 0));
  hipLaunchKernelGGL(k_down_mfma2<D>, dim3(cov->n_leaves, (unsigned)((nrhs + 255) / 256)),
                     dim3(512), 0, st, cov->leaf_off.p, cov->pts.p, n, cov->cheb.p, cov->fc.p,
                     cov->anc_ptr.p, cov->anc_idx.p, ws.yhat, sp ? cov->sp_ynz.p : nullptr,
                     cov->perm.p, nrhs, sp ? sp->order : nullptr, sp ? sp->j0 : 0, Y, ldy);
}

void apply_multi(fkf_cov *cov, const ApplyWs &ws, int nrhs, double *Y, int64_t ldy,
                 hipStream_t st, const SparseRhs *sp = nullptr) {
  const bool m = cov->mixed;
  if (cov->d == 2)
    m ? apply_multi_t<2, true>(cov, ws, nrhs, Y, ldy, st, sp)
      : apply_multi_t<2, false>(cov, ws, nrhs, Y, ldy, st, sp);
  else
    m ? apply_multi_t<3, true>(cov, ws, nrhs, Y, ldy, st, sp)
      : apply_multi_t<3, false>(cov, ws, nrhs, Y, ldy, st, sp);
}

}  // namespace

namespace {

// Doubles of each workspace region of an nc-column product block: the
// gathered columns xt, and either the one-column near partials and far-field
// vectors or the several-column coefficient vectors and upward partials.
// Regions start on 256-byte boundaries.
inline int64_t ws_round(int64_t x) { return (x + 31) / 32 * 32; }

int64_t ws_doubles(const fkf_cov *cov, int nc) {
  int64_t t = ws_round(cov->n * nc);
  if (nc == 1) {
    t += ws_round(std::max<int64_t>(cov->n_blk, 1) * 128);
    if (cov->n_fc > 0)
      t += 2 * ws_round(cov->n_coef) + ws_round(std::max<int64_t>(cov->n_part_up, 1)) +
           ws_round(std::max<int64_t>(cov->n_part_pair, 1));
  } else if (cov->n_fc > 0) {
    t += 2 * ws_round(cov->n_coef * nc) + ws_round(cov->n_part_up_m * nc);
  }
  return t;
}

// The workspace of an nc-column block laid out from base (ws_doubles(cov, nc)
// doubles of device memory).
ApplyWs ws_carve(const fkf_cov *cov, int nc, double *base) {
  ApplyWs ws{};
  double *q = base;
  auto take = [&](int64_t len) {
    double *r = q;
    q += ws_round(len);
    return r;
  };
  ws.xt = take(cov->n * nc);
  if (nc == 1) {
    ws.part = take(std::max<int64_t>(cov->n_blk, 1) * 128);
    if (cov->n_fc > 0) {
      ws.xhat = take(cov->n_coef);
      ws.yhat = take(cov->n_coef);
      ws.part_up = take(std::max<int64_t>(cov->n_part_up, 1));
      ws.part_pair = take(std::max<int64_t>(cov->n_part_pair, 1));
    }
  } else if (cov->n_fc > 0) {
    ws.xhat = take(cov->n_coef * nc);
    ws.yhat = take(cov->n_coef * nc);
    ws.part_up_m = take(cov->n_part_up_m * nc);
  }
  return ws;
}

// Y = Gamma X in column blocks of at most `chunk` columns; the workspace of
// each block is laid out from `base`, or (base == nullptr) from the handle's
// workspace buffer, grown on demand.
void apply_blocks(fkf_cov *cov, const double *X, int64_t ldx, int32_t nrhs, double *Y,
                  int64_t ldy, int32_t chunk, double *base, hipStream_t st) {
  const int64_t n = cov->n;
  for (int32_t c0 = 0; c0 < nrhs; c0 += chunk) {
    const int32_t nc = std::min(chunk, nrhs - c0);
    const double *Xc = X + ldx * (int64_t)c0;
    double *Yc = Y + ldy * (int64_t)c0;
    if (!base) cov->ws.reserve((size_t)ws_doubles(cov, nc));
    const ApplyWs ws = ws_carve(cov, nc, base ? base : cov->ws.p);
    dim3 gg((unsigned)((n + 255) / 256), (unsigned)nc);
    {
      FKF_TRACE("hmat_gather", st);
      hipLaunchKernelGGL(k_gather, gg, dim3(256), 0, st, Xc, ldx, nc, cov->perm.p, n, ws.xt);
    }
    if (nc == 1) {
      apply_one(cov, ws, Yc, st);
    } else {
      apply_multi(cov, ws, nc, Yc, ldy, st);
    }
    FKF_CHECK_HIP(hipGetLastError());
  }
}

// ---------------------------------------------- allocation-free product ---
// Workspace of fkf_cov_apply_noalloc: one array per device, set up by the
// code object's load and held until the process ends.  Host code must never
// pass `scratch` itself to a kernel (on the host it only names the symbol):
// the device address of each device's copy comes from hipGetSymbolAddress.
constexpr int64_t kScratchBytes = int64_t(64) << 20;
__device__ __align__(256) double scratch[kScratchBytes / 8];

double *scratch_ptr() {
  static std::mutex mu;
  static std::map<int, double *> ptrs;   // per device
  int dev = 0;
  FKF_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = ptrs.find(dev);
  if (it != ptrs.end()) return it->second;
  void *p = nullptr;
  FKF_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error{FKF_E_HIP, "hipGetSymbolAddress returned a null scratch address"};
  ptrs.emplace(dev, static_cast<double *>(p));
  return static_cast<double *>(p);
}

}  // namespace

extern "C" fkf_status fkf_cov_apply(fkf_cov *cov, const double *X, int64_t ldx, int32_t nrhs,
                                    double *Y, int64_t ldy, void *stream) {
  return guarded([&] {
    FKF_REQUIRE(cov != nullptr, "fkf_cov_apply: NULL handle");
    FKF_REQUIRE(nrhs >= 0, "fkf_cov_apply: nrhs < 0");
    if (nrhs == 0) return;
    FKF_REQUIRE(X != nullptr && Y != nullptr, "fkf_cov_apply: NULL array");
    FKF_REQUIRE(ldx >= cov->n && ldy >= cov->n, "fkf_cov_apply: leading dimension < n");
    // the several-column workspaces (gathered columns, coefficient vectors,
    // upward partials) grow with the number of columns: apply in column
    // blocks that keep them within the bound (at least 2 columns a block)
    const int64_t budget = cov->hp.workspace_bytes > 0 ? cov->hp.workspace_bytes
                                                        : (int64_t(16) << 30);
    const int64_t per_col = 8 * (cov->n + 2 * cov->n_coef + cov->n_part_up_m);
    const int32_t chunk =
        nrhs == 1 ? 1 : (int32_t)std::min<int64_t>(nrhs, std::max<int64_t>(2, budget / per_col));
    apply_blocks(cov, X, ldx, nrhs, Y, ldy, chunk, nullptr, as_stream(stream));
  });
}

extern "C" fkf_status fkf_cov_apply_noalloc(fkf_cov *cov, const double *X, int64_t ldx,
                                            int32_t nrhs, double *Y, int64_t ldy,
                                            void *stream) {
  return guarded([&] {
    FKF_REQUIRE(cov != nullptr, "fkf_cov_apply_noalloc: NULL handle");
    FKF_REQUIRE(nrhs >= 0, "fkf_cov_apply_noalloc: nrhs < 0");
    if (nrhs == 0) return;
    FKF_REQUIRE(X != nullptr && Y != nullptr, "fkf_cov_apply_noalloc: NULL array");
    FKF_REQUIRE(ldx >= cov->n && ldy >= cov->n, "fkf_cov_apply_noalloc: leading dimension < n");
    const int64_t cap = kScratchBytes / 8;
    const int64_t one = ws_doubles(cov, 1);
    if (one > cap)
      throw Error{FKF_E_ARG, "fkf_cov_apply_noalloc: the one-column workspace of this operator (" +
                                 std::to_string((one * 8) >> 20) +
                                 " MiB) exceeds the fixed scratch of " +
                                 std::to_string(kScratchBytes >> 20) + " MiB"};
    // widest column block whose workspace fits the scratch (one column at a
    // time when not even two fit)
    int32_t chunk = 1;
    if (nrhs > 1 && ws_doubles(cov, 2) <= cap) {
      int32_t lo = 2, hi = nrhs;
      while (lo < hi) {
        const int32_t mid = lo + (hi - lo + 1) / 2;
        if (ws_doubles(cov, mid) <= cap) lo = mid;
        else hi = mid - 1;
      }
      chunk = lo;
    }
    apply_blocks(cov, X, ldx, nrhs, Y, ldy, chunk, scratch_ptr(), as_stream(stream));
  });
}

namespace fkf {

bool cov_apply_sparse_rows(fkf_cov *cov, int n_m, const int64_t *rowptr, const int32_t *col,
                           const double *val, int64_t nnz, int64_t max_row, const int32_t *order,
                           double *Y, int64_t ldy, hipStream_t st) {
  if (!cov->sp_ok || cov->n_fc == 0 || n_m < 2 || max_row > kSpRowMax) return false;
  cov->sp_tix.reserve((size_t)std::max<int64_t>(nnz, 1));
  cov->sp_val.reserve((size_t)std::max<int64_t>(nnz, 1));
  // column blocks within the workspace bound, as in the dense product (here
  // the two coefficient vectors and the per-leaf counts of each column; at
  // most 4 * 65535 columns for the grids)
  const int64_t budget = cov->hp.workspace_bytes > 0 ? cov->hp.workspace_bytes
                                                      : (int64_t(16) << 30);
  const int64_t per_col = 8 * 2 * cov->n_coef + 4 * (cov->n_leaves + 1);
  int32_t chunk = (int32_t)std::min<int64_t>(
      {(int64_t)n_m, std::max<int64_t>(2, budget / per_col), int64_t(4) * 65535});
  while (chunk > 2 && n_m % chunk == 1) --chunk;   // no block of a single column
  cov->sp_cnt.reserve((size_t)std::min(chunk, n_m) * (cov->n_leaves + 1));
  // the coefficient vectors of a block (no gathered columns, no upward partials)
  const int64_t coef = ws_round(cov->n_coef * std::min(chunk, n_m));
  cov->ws.reserve((size_t)(2 * coef));
  ApplyWs ws{};
  ws.xhat = cov->ws.p;
  ws.yhat = cov->ws.p + coef;
  for (int32_t c0 = 0; c0 < n_m; c0 += chunk) {
    const int32_t nc = std::min(chunk, n_m - c0);
    hipLaunchKernelGGL(k_sparse_rows, dim3((unsigned)nc), dim3(256), 0, st, rowptr, col, val,
                       cov->iperm.p, cov->leaf_off.p, cov->n_leaves, c0, order, cov->sp_tix.p,
                       cov->sp_val.p, cov->sp_cnt.p);
    const SparseRhs sp{rowptr, c0, order};
    apply_multi(cov, ws, nc, Y, ldy, st, &sp);
    FKF_CHECK_HIP(hipGetLastError());
  }
  return true;
}

}  // namespace fkf

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
    info->near_bytes = cov->n_blk * 4096 * (int64_t)(cov->mixed ? sizeof(float) : sizeof(double));
    info->far_bytes =
        cov->stored ? cov->n_kst * (int64_t)(cov->mixed ? sizeof(float) : sizeof(double)) : 0;
    info->far_coef_per_rhs = cov->n_coef;
    info->far_interp_entries = cov->n_interp;
    info->far_pair_entries = cov->n_kpair;
    info->coupling_groups = cov->grouped ? cov->n_grp_groups : 0;
    info->coupling_items = cov->grouped ? cov->n_grp_items : 0;
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
    FKF_REQUIRE(hp->precision == FKF_FP64 || hp->precision == FKF_MIXED,
                "fkf_cov_plan: unknown precision");
    FKF_REQUIRE(hp->far_eval == 0 || hp->far_eval == 1, "fkf_cov_plan: far_eval must be 0 or 1");
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
    int64_t nk = 0, nk_all = 0;
    {
      // as at build: one stored matrix per distinct pair geometry
      std::vector<char> isf(t.nodes.size(), 0);
      for (auto &pr : far) isf[pr.first] = isf[pr.second] = 1;
      std::vector<double> ctr(t.nodes.size() * kMaxDim, 0.0), hw(t.nodes.size() * kMaxDim, 0.0);
      std::vector<const double *> cs, hs;
      for (size_t nd = 0; nd < t.nodes.size(); ++nd) {
        for (int k = 0; k < d; ++k) {
          ctr[nd * kMaxDim + k] = 0.5 * (t.nodes[nd].lo[k] + t.nodes[nd].hi[k]);
          hw[nd * kMaxDim + k] = 0.5 * (t.nodes[nd].hi[k] - t.nodes[nd].lo[k]);
        }
        if (isf[nd]) {
          cs.push_back(&ctr[nd * kMaxDim]);
          hs.push_back(&hw[nd * kMaxDim]);
        }
      }
      const double q = coupling_quantum(d, cs, hs);
      // one stored matrix per geometry of an ordered pair (target, partner),
      // keyed as at build with the partner's nodes as rows
      std::map<std::vector<int64_t>, int> shapes;
      for (auto &pr : far) {
        cov += t.nodes[pr.first].size() * t.nodes[pr.second].size();
        const int pt = lp[t.nodes[pr.first].level], pp = lp[t.nodes[pr.second].level];
        int64_t a = 1, b = 1;
        for (int k = 0; k < d; ++k) {
          a *= pt;
          b *= pp;
        }
        if (pr.first < pr.second) nk_all += a * b;
        const size_t i = (size_t)pr.second * kMaxDim, j = (size_t)pr.first * kMaxDim;
        if (shapes.emplace(coupling_key(d, pp, pt, &ctr[i], &hw[i], &ctr[j], &hw[j], q), 0).second)
          nk += a * b;
      }
    }
    info->far_pair_entries = nk_all;
    {
      std::vector<char> is_far(t.nodes.size(), 0);
      for (auto &pr : far) is_far[pr.first] = is_far[pr.second] = 1;
      int64_t coef = 0, interp = 0;
      for (size_t nd = 0; nd < t.nodes.size(); ++nd)
        if (is_far[nd]) {
          int64_t pd = 1;
          for (int k = 0; k < d; ++k) pd *= lp[t.nodes[nd].level];
          coef += pd;
          interp += t.nodes[nd].size() * pd;
        }
      info->far_coef_per_rhs = coef;
      info->far_interp_entries = interp;
    }
    const int64_t kb = nk * (int64_t)(hp->precision == FKF_MIXED ? sizeof(float) : sizeof(double));
    info->far_bytes = (kb <= kMaxCouplingBytes && hp->far_eval == 0) ? kb : 0;
    info->n_near_blocks = nb;
    info->n_near_pairs = (int64_t)near.size();
    info->n_far_pairs = (int64_t)far.size();
    info->near_bytes =
        nb * 4096 * (int64_t)(hp->precision == FKF_MIXED ? sizeof(float) : sizeof(double));
    info->covered_entries = cov;
    for (int l = 0; l < 32 && l < (int)lp.size(); ++l) info->cheb_p[l] = lp[l];
  });
}

namespace fkf {
double cov_variance(const fkf_cov *cov) {
  return cov->kind >= FKF_MATERN_12_DLENGTH ? 0.0 : cov->theta;   // diagonal of the operator
}
int cov_kind(const fkf_cov *cov) { return cov->kind; }
double cov_length(const fkf_cov *cov) { return cov->ell; }
bool cov_mixed(const fkf_cov *cov) { return cov->mixed; }
int64_t cov_n(const fkf_cov *cov) { return cov->n; }
}  // namespace fkf
