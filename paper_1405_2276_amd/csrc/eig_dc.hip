// Symmetric FP64 eigensolver for one dense problem of order 3..1024: the
// projected eigenproblem of the generalized eigenvalue problem (Section
// 2.2.2) and the small symmetric problems of the low-rank updates (Section
// 2.4, Algorithm 5).  Three stages:
//
//  1. Householder reduction to tridiagonal form T = Q^T A Q in one launch.
//     The columns of A are dealt cyclically to G workgroups and stay in
//     their registers for the whole reduction; each reflector step is one
//     exchange between the workgroups, in which every workgroup publishes
//     p = S v for its own columns and the owner of the next pivot column
//     publishes that column (each double as two tagged 64-bit words, read
//     by polling until the tags match).  Every workgroup then forms w, the
//     updated pivot column and the next reflector itself (identical
//     arithmetic in every workgroup), and applies the rank-2 update to its
//     columns fused with the next step's p.
//  2. Divide and conquer on T (Cuppen's splitting into halves coupled by a
//     rank-one term, down to 1 x 1 leaves).  A merge sorts the children's
//     eigenvalues, deflates tiny components of the coupling vector and
//     nearly equal eigenvalues (plane rotations), finds each remaining root
//     of the secular equation 1 + rho sum z_j^2 / (d_j - lambda) = 0 by a
//     two-pole rational model safeguarded by bisection on the lattice of
//     doubles (origin at the nearer pole so that every d_j - lambda is
//     formed without cancellation), recomputes z from the roots by the
//     Gu-Eisenstat product formula so that the eigenvectors
//     z_i / (d_i - lambda_j) are numerically orthogonal, and multiplies them
//     into the children's eigenvectors on the FP64 matrix cores.  All merges
//     of one tree height form one launch per phase.
//  3. Back-transformation of T's eigenvectors by the reflectors, written in
//     descending eigenvalue order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.h"
#include "linalg.h"
#include "trace.h"

namespace fkf {
namespace {

constexpr int kTrThreads = 512;
constexpr long kSpinMax = 1L << 24;  // polls of an exchange before it is declared failed
constexpr int kDcMaxN = 1024;        // largest order of this solver
constexpr int kKR = kDcMaxN / 64;    // secular terms per lane

typedef double v4d __attribute__((ext_vector_type(4)));

// Sum over the 512 threads of a workgroup in a fixed order; every thread
// gets the result.  red: 8 doubles of LDS, whose previous readers must have
// passed a barrier since (the callers alternate two such buffers).
__device__ double block_sum512(double v, double *red) {
  v = wave_sum_all(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += red[i];
  return s;
}

// Reflector H = I - tau v v^T with v[r0] = 1 and v = 0 above r0, mapping
// x = cc[r0..n) to (beta, 0, ..., 0): beta = -sign(x0) ||x||, tau = (beta -
// x0) / beta, v[i] = x[i] / (x0 - beta) below r0; tau = 0 and beta = x0 when
// x has nothing below x0.  Writes v (n entries) to LDS; the caller
// synchronises before reading it.
__device__ void householder(const double *cc, int r0, int n, double *v, double *red, double &tau,
                            double &beta) {
  double s = 0.0;
  for (int i = r0 + 1 + threadIdx.x; i < n; i += kTrThreads) s = fma(cc[i], cc[i], s);
  const double xn2 = block_sum512(s, red);
  const double x0 = cc[r0];
  double scale = 0.0;
  if (xn2 == 0.0) {
    tau = 0.0;
    beta = x0;
  } else {
    beta = -copysign(sqrt(fma(x0, x0, xn2)), x0);
    tau = (beta - x0) / beta;
    scale = 1.0 / (x0 - beta);
  }
  for (int i = threadIdx.x; i < n; i += kTrThreads)
    v[i] = i < r0 ? 0.0 : (i == r0 ? 1.0 : cc[i] * scale);
}

// Tagged exchange words: a double travels as two 64-bit words (low half,
// high half), each with the step tag in its upper 32 bits, written and read
// as single relaxed agent-scope atomics.  A reader accepts a value once both
// words carry the tag it waits for, so no fence orders data and flags.
__device__ __forceinline__ void put_tagged(unsigned long long *w, double v, unsigned int tag) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned long long t = (unsigned long long)tag << 32;
  __hip_atomic_store(w, t | (b & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 1, t | (b >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool get_tagged(unsigned long long *w, unsigned int tag, double &v) {
  const unsigned long long lo = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long hi =
      __hip_atomic_load(w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((unsigned int)(lo >> 32) != tag || (unsigned int)(hi >> 32) != tag) return false;
  v = __longlong_as_double((long long)(((hi & 0xffffffffull) << 32) | (lo & 0xffffffffull)));
  return true;
}

// Householder tridiagonalization (stage 1), G workgroups of 512 threads;
// workgroup g owns columns j = c G + g (c < 8 CW) of A: wavefront w holds
// its columns c = w + 8 q (q < CW) in registers, lane l the rows l + 64 m
// (m < RM, n <= 64 RM).  The n-vectors v, w and the pivot column live in
// LDS.  Outputs: d (n), e (n - 1), the reflectors hv (column k = v_k, n x n)
// and tau (n - 2).
//
// Exchange of step k (tag k + 1, words xw + 4 n (k & 1), zero at launch):
// entry j of p' = S v_k from the owner of column j (words 2 j, 2 j + 1) and
// the pivot column k + 1 from its owner (words 2 n + 2 i, 2 n + 2 i + 1),
// written as soon as they are formed; each thread waits for the entries of
// its rows.  A thread that waits longer than kSpinMax polls sets the failure
// flag fail[0] (0 at launch), and every workgroup leaves at its next check.
template <int RM, int CW>
__global__ void __launch_bounds__(kTrThreads) k_tridiag(const double *__restrict__ A, int64_t lda,
                                                        int n, int G,
                                                        double *__restrict__ hv,
                                                        double *__restrict__ htau,
                                                        double *__restrict__ dg,
                                                        double *__restrict__ eg,
                                                        unsigned long long *__restrict__ xw,
                                                        int *__restrict__ fail) {
  constexpr int NP = 64 * RM, NR = (NP + kTrThreads - 1) / kTrThreads;
  __shared__ double vecs[4 * NP];
  double *vv = vecs, *vn = vv + NP, *ww = vn + NP, *cc = ww + NP;
  __shared__ double red[16];   // two reduction buffers, used in turn
  __shared__ double pk1s;
  __shared__ int bad;
  const int g = blockIdx.x, tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  double a[CW][RM];
  int jq[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) {
    const int j = (wv + 8 * q) * G + g;
    jq[q] = j < n ? j : -1;
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int i = lane + 64 * m;
      a[q][m] = (j < n && i < n) ? A[i + lda * j] : 0.0;
    }
  }
  for (int i = tid; i < n; i += kTrThreads) cc[i] = A[i];
  if (tid == 0) bad = 0;
  __syncthreads();
  double tau, beta;
  householder(cc, 1, n, vv, red, tau, beta);
  if (g == 0 && tid == 0) {
    dg[0] = cc[0];
    eg[0] = beta;
    htau[0] = tau;
  }
  __syncthreads();
  if (g == 0)
    for (int i = tid; i < n; i += kTrThreads) __builtin_nontemporal_store(vv[i], hv + i);

  // Own columns j >= k + 2: rank-2 update of step k (when upd; v and w vanish
  // on rows <= k, so every row is updated) and p'_j = S[:, j] . v_{k+1} for
  // the next step (vnext, zero on rows <= k + 1), published with the pivot
  // column k + 2 (by its owner) into exchange k + 1.  At the last step
  // (vnext null) the owner of column n - 1 writes d[n - 1].
  auto fused = [&](int k, bool upd, const double *vnext) {
    const int jmin = k + 2;
    unsigned long long *x = xw + (size_t)((k + 1) & 1) * 4 * n;
    const unsigned int tag = (unsigned int)(k + 2);
    double vr[RM], wr[RM], nr[RM];
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int i = lane + 64 * m;
      vr[m] = (upd && i < n) ? vv[i] : 0.0;
      wr[m] = (upd && i < n) ? ww[i] : 0.0;
      nr[m] = (vnext && i < n) ? vnext[i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      const int j = jq[q];
      if (j < jmin) continue;   // also j = -1 (no column)
      const double wj = upd ? ww[j] : 0.0, vj = upd ? vv[j] : 0.0;
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        double y = fma(-vr[m], wj, a[q][m]);
        y = fma(-wr[m], vj, y);
        a[q][m] = y;
        acc = fma(y, nr[m], acc);
      }
      if (vnext) {
        acc = wave_sum_all(acc);
        if (lane == 0) put_tagged(x + 2 * j, acc, tag);
        if (j == jmin) {
#pragma unroll
          for (int m = 0; m < RM; ++m) {
            const int i = lane + 64 * m;
            if (i >= jmin && i < n) put_tagged(x + 2 * n + 2 * i, a[q][m], tag);
          }
        }
      } else if (j == n - 1) {
#pragma unroll
        for (int m = 0; m < RM; ++m)
          if (lane + 64 * m == n - 1) dg[n - 1] = a[q][m];
      }
    }
  };
  fused(-1, false, vv);

  for (int k = 0; k <= n - 3; ++k) {
    unsigned long long *x = xw + (size_t)(k & 1) * 4 * n;
    const unsigned int tag = (unsigned int)(k + 1);
    // this thread's rows i = tid + 512 r: p_i and the pivot column entry
    double pr[NR], cr[NR], vr[NR];
    double part = 0.0;
    bool late = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = tid + kTrThreads * r;
      const bool in = i > k && i < n;
      pr[r] = 0.0;
      cr[r] = 0.0;
      if (in) {
        bool gp = false, gc = false;
        long polls = 0;
        for (;;) {
          if (!gp) gp = get_tagged(x + 2 * i, tag, pr[r]);
          if (!gc) gc = get_tagged(x + 2 * n + 2 * i, tag, cr[r]);
          if (gp && gc) break;
          if (++polls > kSpinMax ||
              ((polls & 63) == 0 && __hip_atomic_load(fail, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT) != 0)) {
            __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            late = true;
            break;
          }
        }
        if (i == k + 1) pk1s = pr[r];
      }
      vr[r] = in ? vv[i] : 0.0;
      part = fma(pr[r], vr[r], part);
    }
    if (late) bad = 1;
    // p = tau S v, w = p - (tau / 2)(p . v) v; every thread needs w[k + 1]
    const double pv = block_sum512(part, red);
    if (bad) return;
    const double kc = 0.5 * tau * tau * pv;
    const double wk1 = fma(-kc, 1.0, tau * pk1s);   // v[k + 1] = 1
    const bool more = k + 1 <= n - 3;
    double npart = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = tid + kTrThreads * r;
      if (i < n) {
        const double w_i = i > k ? fma(-kc, vr[r], tau * pr[r]) : 0.0;
        ww[i] = w_i;
        // pivot column k + 1 after step k
        cr[r] = i > k ? fma(-vr[r], wk1, cr[r]) - w_i : 0.0;
        cc[i] = cr[r];
        if (i > k + 2) npart = fma(cr[r], cr[r], npart);
      }
    }
    const double xn2 = block_sum512(npart, red + 8);   // also orders the LDS writes
    double tau_n = 0.0, beta_n = 0.0;
    if (more) {
      // reflector k + 1 from the pivot column below its diagonal
      const double x0 = cc[k + 2];
      double scale = 0.0;
      if (xn2 == 0.0) {
        beta_n = x0;
      } else {
        beta_n = -copysign(sqrt(fma(x0, x0, xn2)), x0);
        tau_n = (beta_n - x0) / beta_n;
        scale = 1.0 / (x0 - beta_n);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int i = tid + kTrThreads * r;
        if (i < n) {
          const double v = i < k + 2 ? 0.0 : (i == k + 2 ? 1.0 : cr[r] * scale);
          vn[i] = v;
          if (g == 0) __builtin_nontemporal_store(v, hv + (size_t)(k + 1) * n + i);
        }
      }
      if (g == 0 && tid == 0) {
        dg[k + 1] = cc[k + 1];
        eg[k + 1] = beta_n;
        htau[k + 1] = tau_n;
      }
    } else if (g == 0 && tid == 0) {
      dg[n - 2] = cc[n - 2];
      eg[n - 2] = cc[n - 1];
    }
    __syncthreads();
    fused(k, true, more ? vn : nullptr);
    double *t = vv;
    vv = vn;
    vn = t;
    tau = tau_n;
  }
}

// ------------------------------------------------ divide and conquer ---
// A merge node covers indices [off, off + s) of T, split at off + m.  Per
// node the working arrays use the same index range: lam (eigenvalues,
// ascending), Qc (eigenvectors, the diagonal block of an n x n array), and
// for the merge itself Qp (sorted and deflation-rotated children's
// eigenvectors, the k secular columns first), dd/zz (the k remaining poles
// and coupling components), dv (candidate eigenvalues in Qp column order),
// dels (d_j - lambda_i, k x k), zh (recomputed z), U (k x k eigenvectors of
// the rank-one problem), csrc (Qp column of each output column), kk[off] = k
// and rho[off].

// Diagonal of the leaves: every coupling e_i is a split point, so leaf i is
// d_i - |e_{i-1}| - |e_i|, with eigenvector 1.
__global__ void k_dc_leaves(const double *__restrict__ dg, const double *__restrict__ eg, int n,
                            double *__restrict__ lam, double *__restrict__ Qc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = dg[i];
  if (i > 0) d -= fabs(eg[i - 1]);
  if (i < n - 1) d -= fabs(eg[i]);
  lam[i] = d;
  Qc[i + (int64_t)n * i] = 1.0;
}

struct DcNode {
  int32_t off, s, m, pad;
};

// Device arrays of the merges (indexed by the node's range [off, off + s)):
// qsrc[off + u] = child column of Qp column u; rot_x/rot_y/rot_c/rot_s[off +
// q] the deflation rotations (Qp columns, cosine, sine) in order and
// nrot[off] their number.
struct DcArrays {
  double *lam, *Qc, *Qp, *U, *dels, *dd, *zz, *dv, *zh, *rho, *rot_c, *rot_s;
  int *kk, *csrc, *qsrc, *rot_x, *rot_y, *nrot;
};

constexpr int kPrepThreads = 256;

__device__ double block_max256(double v, double *red) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v = fmax(v, __shfl_xor(v, m));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__device__ double block_sum256(double v, double *red) {
  v = wave_sum_all(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Exclusive prefix count of flags f[0..s) (0/1) into pos[0..s); returns the
// total.  cnt: kPrepThreads + 1 ints of LDS.  Each thread counts a run of
// consecutive flags; the runs are scanned across lanes and wavefronts.
__device__ int block_scan256(const int *f, int s, int *pos, int *cnt) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int per = (s + kPrepThreads - 1) / kPrepThreads;
  const int b = tid * per, e = min(s, b + per);
  int c = 0;
  for (int t = b; t < e; ++t) c += f[t];
  int incl = c;   // inclusive scan within the wavefront
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d);
    if (lane >= d) incl += y;
  }
  __syncthreads();
  if (lane == 63) cnt[wv] = incl;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wv; ++w) base += cnt[w];
  const int total = cnt[0] + cnt[1] + cnt[2] + cnt[3];
  int run = base + incl - c;
  for (int t = b; t < e; ++t) {
    pos[t] = run;
    run += f[t];
  }
  __syncthreads();
  return total;
}

// Merge preparation, one workgroup per node: coupling vector z (last row of
// the left child's eigenvectors, sign(beta) times the first row of the
// right child's), normalised with rho = |beta| ||z||^2; the children's
// eigenvalues merged into ascending order; deflation of components with
// rho |z_j| <= tol and of nearly equal neighbours (rotation when
// |t c s| <= tol, t the gap), tol = 8 eps max(max |d|, max |z|); then Qp,
// dd, zz, dv, kk, rho.  The neighbour test is evaluated for all pairs at
// once on the unrotated values; only when some pair deflates does one
// thread rescan in order (each rotation changes the next comparison).
__global__ void __launch_bounds__(kPrepThreads) k_dc_prep(const DcNode *__restrict__ nodes, int n,
                                                         const double *__restrict__ eg,
                                                         DcArrays ar) {
  const double *__restrict__ lam = ar.lam;
  const double *__restrict__ Qc = ar.Qc;
  __shared__ double L0[kDcMaxN], Z0[kDcMaxN], Ds[kDcMaxN], Zs[kDcMaxN];
  __shared__ int perm[kDcMaxN], keep[kDcMaxN], pos[kDcMaxN], col[kDcMaxN];
  __shared__ int rp[kDcMaxN], rj[kDcMaxN], trig[kDcMaxN];
  __shared__ double rc[kDcMaxN], rs[kDcMaxN];
  __shared__ double red[4];
  __shared__ int cnt[kPrepThreads + 1];
  __shared__ int nrot, any_close;
  const DcNode nd = nodes[blockIdx.x];
  const int off = nd.off, s = nd.s, m = nd.m, tid = threadIdx.x;
  const double beta = eg[off + m - 1];
  const double sg = beta >= 0.0 ? 1.0 : -1.0;
  double zs = 0.0;
  for (int t = tid; t < s; t += kPrepThreads) {
    L0[t] = lam[off + t];
    const double z = t < m ? Qc[(off + m - 1) + (int64_t)n * (off + t)]
                           : sg * Qc[(off + m) + (int64_t)n * (off + t)];
    Z0[t] = z;
    zs = fma(z, z, zs);
  }
  const double zn2 = block_sum256(zs, red);
  const double zinv = 1.0 / sqrt(zn2);
  const double rho = fabs(beta) * zn2;
  // merge of the two ascending lists (ties: left child first)
  for (int t = tid; t < s; t += kPrepThreads) {
    const double x = L0[t];
    int lo, hi;
    if (t < m) {   // count right-list entries < x
      lo = m;
      hi = s;
      while (lo < hi) {
        const int md = (lo + hi) >> 1;
        if (L0[md] < x) lo = md + 1; else hi = md;
      }
      const int r = t + (lo - m);
      perm[r] = t;
    } else {       // count left-list entries <= x
      lo = 0;
      hi = m;
      while (lo < hi) {
        const int md = (lo + hi) >> 1;
        if (L0[md] <= x) lo = md + 1; else hi = md;
      }
      const int r = (t - m) + lo;
      perm[r] = t;
    }
  }
  __syncthreads();
  double dmax = 0.0, zmax = 0.0;
  for (int r = tid; r < s; r += kPrepThreads) {
    const int t = perm[r];
    Ds[r] = L0[t];
    Zs[r] = Z0[t] * zinv;
    dmax = fmax(dmax, fabs(Ds[r]));
    zmax = fmax(zmax, fabs(Zs[r]));
  }
  const double tol = 8.0 * 2.220446049250313e-16 * fmax(block_max256(dmax, red), block_max256(zmax, red));
  // component test, then the neighbour test on unrotated values
  for (int r = tid; r < s; r += kPrepThreads) keep[r] = rho * fabs(Zs[r]) > tol ? 1 : 0;
  if (tid == 0) {
    nrot = 0;
    any_close = 0;
  }
  __syncthreads();
  const int nk = block_scan256(keep, s, pos, cnt);   // pos[r]: index among kept
  for (int r = tid; r < s; r += kPrepThreads)
    if (keep[r]) col[pos[r]] = r;                    // kept positions in order
  __syncthreads();
  // trig[u]: the pair (col[u - 1], col[u]) deflates on unrotated values
  for (int u = tid; u < nk; u += kPrepThreads) {
    int t = 0;
    if (u > 0) {
      const int p = col[u - 1], j = col[u];
      const double sv = Zs[p], cv = Zs[j];
      const double ta = hypot(cv, sv);
      const double c = cv / ta, sn = -sv / ta;
      t = fabs((Ds[j] - Ds[p]) * c * sn) <= tol ? 1 : 0;
    }
    trig[u] = t;
    if (t) any_close = 1;
  }
  __syncthreads();
  if (any_close && tid == 0) {
    // in order: a pair is re-tested on current values only when the pair
    // before it rotated (which changed its left element); otherwise the
    // unrotated test stands
    bool rotated = false;
    int q = 0;
    for (int u = 1; u < nk; ++u) {
      if (!rotated && !trig[u]) continue;
      const int p = col[u - 1], j = col[u];
      const double sv = Zs[p], cv = Zs[j];
      const double ta = hypot(cv, sv);
      const double c = cv / ta, sn = -sv / ta;
      rotated = fabs((Ds[j] - Ds[p]) * c * sn) <= tol;
      if (rotated) {
        Zs[j] = ta;
        Zs[p] = 0.0;
        rp[q] = p;
        rj[q] = j;
        rc[q] = c;
        rs[q] = sn;
        ++q;
        const double dp = Ds[p] * c * c + Ds[j] * sn * sn;
        const double dj = Ds[p] * sn * sn + Ds[j] * c * c;
        Ds[p] = dp;
        Ds[j] = dj;
        keep[p] = 0;
      }
    }
    nrot = q;
  }
  __syncthreads();
  const int k = any_close ? block_scan256(keep, s, pos, cnt) : nk;
  // Qp column of sorted position r: kept ones first (in order), then the
  // deflated ones (in order)
  for (int r = tid; r < s; r += kPrepThreads) col[r] = keep[r] ? pos[r] : k + (r - pos[r]);
  __syncthreads();
  for (int r = tid; r < s; r += kPrepThreads) {
    const int u = col[r];
    ar.qsrc[off + u] = perm[r];
    if (u < k) {
      ar.dd[off + u] = Ds[r];
      ar.zz[off + u] = Zs[r];
    } else {
      ar.dv[off + u] = Ds[r];
    }
  }
  const int nr = any_close ? nrot : 0;
  for (int q = tid; q < nr; q += kPrepThreads) {
    ar.rot_x[off + q] = col[rp[q]];
    ar.rot_y[off + q] = col[rj[q]];
    ar.rot_c[off + q] = rc[q];
    ar.rot_s[off + q] = rs[q];
  }
  if (tid == 0) {
    ar.kk[off] = k;
    ar.rho[off] = rho;
    ar.nrot[off] = nr;
  }
}

// One 64-lane wavefront per (node, root i) of the secular equation f(tau) =
// 1 + sum_j z2_j / (delta_j - tau) = 0, tau = lambda_i - d_o in the frame of
// the nearer pole o (delta_j = d_j - d_o; the root lies between the poles i
// and i + 1, or above the last pole).  Iterates of a two-pole rational model
// (the sums over the poles left and right of the root are matched in value
// and slope by a / (pole - tau) + b, and the model's root in the interval is
// taken), safeguarded by a bracket kept from the signs of f and bisection on
// the lattice of doubles whenever a step leaves the bracket or the model
// stalls.  Then dels[j][i] = delta_j - tau and dv[i] = d_o + tau.
__device__ __forceinline__ double lattice_mid_pos(double lo, double hi) {
  const long long a = __double_as_longlong(lo), b = __double_as_longlong(hi);
  return __longlong_as_double(a + ((b - a) >> 1));
}

// midpoint on the lattice of [lo, hi] (both >= 0 or both <= 0)
__device__ __forceinline__ double lattice_mid(double lo, double hi) {
  return lo >= 0.0 ? lattice_mid_pos(lo, hi) : -lattice_mid_pos(0.0 - hi, 0.0 - lo);
}

__global__ void __launch_bounds__(256) k_dc_secular(const DcNode *__restrict__ nodes,
                                                    const int2 *__restrict__ wmap, int nw, int n,
                                                    DcArrays ar) {
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (q >= nw) return;
  const int2 wm = wmap[q];
  const DcNode nd = nodes[wm.x];
  const int off = nd.off, i = wm.y;
  {
    // Qp column i: the children's eigenvector it comes from, zero outside
    // that child's rows (block diagonal)
    const int t = ar.qsrc[off + i];
    const double *src = ar.Qc + off + (int64_t)n * (off + t);
    double *dst = ar.Qp + off + (int64_t)n * (off + i);
    for (int r = lane; r < nd.s; r += 64) dst[r] = ((t < nd.m) == (r < nd.m)) ? src[r] : 0.0;
  }
  const double *__restrict__ dd = ar.dd;
  const double *__restrict__ zz = ar.zz;
  double *__restrict__ dels = ar.dels;
  double *__restrict__ dv = ar.dv;
  const int k = ar.kk[off];
  if (i >= k) return;
  const double *rho_in = ar.rho;
  const double rho = rho_in[off];
  double z2[kKR], bs[kKR];
  double zsum = 0.0;
#pragma unroll
  for (int r = 0; r < kKR; ++r) {
    const int j = lane + 64 * r;
    const bool in = j < k;
    const double z = in ? zz[off + j] : 0.0;
    z2[r] = rho * z * z;
    bs[r] = in ? dd[off + j] : 0.0;
    zsum += z2[r];
  }
  zsum = wave_sum_all(zsum);
  const double di = dd[off + i];
  const bool last = i == k - 1;
  int o = i;
  double lo = 0.0, hi = zsum;
  if (!last) {
    // which half of (d_i, d_{i+1}) holds the root: f at the midpoint
    const double mid = 0.5 * (dd[off + i + 1] - di);
    double f = 0.0;
#pragma unroll
    for (int r = 0; r < kKR; ++r)
      if (lane + 64 * r < k) f += z2[r] / ((bs[r] - di) - mid);
    if (1.0 + wave_sum_all(f) >= 0.0) {
      hi = mid;
    } else {
      o = i + 1;
      lo = -mid;
      hi = 0.0;
    }
  }
  const double dor = dd[off + o];
#pragma unroll
  for (int r = 0; r < kKR; ++r) bs[r] -= dor;   // delta_j
  const double dL = di - dor;                   // pole i in this frame
  const double dR = last ? 0.0 : dd[off + i + 1] - dor;
  double tau = 0.5 * (lo + hi);
  if (tau == 0.0 || tau == lo || tau == hi) tau = lattice_mid(lo, hi);
  for (int it = 0; it < 100; ++it) {
    // f and its slope, split into the poles j <= i and j > i
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
#pragma unroll
    for (int r = 0; r < kKR; ++r) {
      const int j = lane + 64 * r;
      if (j < k) {
        const double del = bs[r] - tau;
        const double t1 = z2[r] / del;
        const double t2 = t1 / del;
        if (j <= i) {
          a0 += t1;
          a1 += t2;
        } else {
          b0 += t1;
          b1 += t2;
        }
      }
    }
    const double psi = wave_sum_all(a0), dpsi = wave_sum_all(a1);
    const double phi = wave_sum_all(b0), dphi = wave_sum_all(b1);
    const double f = 1.0 + psi + phi;
    // f is zero to within its rounding error (terms of psi are negative,
    // those of phi positive)
    if (fabs(f) <= 16.0 * 2.220446049250313e-16 * (1.0 + phi - psi)) break;
    if (f > 0.0) hi = tau; else lo = tau;
    // model step
    const double DL = dL - tau;
    double eta;
    bool ok = false;
    if (last) {
      const double c = f - DL * dpsi;
      if (c > 0.0) {
        eta = DL + DL * DL * dpsi / c;
        ok = true;
      }
    } else {
      const double DR = dR - tau;
      const double BP = DL * DL * dpsi, BF = DR * DR * dphi;
      const double c = f - DL * dpsi - DR * dphi;
      const double a = c * (DL + DR) + BP + BF;
      const double b = c * DL * DR + BP * DR + BF * DL;
      if (c == 0.0) {
        if (a != 0.0) {
          eta = b / a;
          ok = true;
        }
      } else {
        const double sq = sqrt(fmax(a * a - 4.0 * b * c, 0.0));
        const double den = a >= 0.0 ? a + sq : a - sq;
        const double r1 = den / (2.0 * c), r2 = den != 0.0 ? 2.0 * b / den : r1;
        const bool in1 = r1 > DL && r1 < DR, in2 = r2 > DL && r2 < DR;
        if (in2) {
          eta = r2;
          ok = true;
        } else if (in1) {
          eta = r1;
          ok = true;
        }
      }
    }
    const double bis = lattice_mid(lo, hi);
    if (bis == lo || bis == hi) break;   // bracket down to adjacent doubles
    double tn = ok ? tau + eta : bis;
    if (!(tn > lo && tn < hi) || it >= 12) tn = bis;
    const bool done = ok && fabs(tn - tau) <= 2.0 * 2.220446049250313e-16 * fabs(tn);
    tau = tn;
    if (done) break;
  }
#pragma unroll
  for (int r = 0; r < kKR; ++r) {
    const int j = lane + 64 * r;
    if (j < k) dels[(off + j) + (int64_t)n * (off + i)] = bs[r] - tau;
  }
  if (lane == 0) dv[off + i] = dor + tau;
}

// One wavefront per (node, i): zh_i = sign(z_i) sqrt(|(lambda_i - d_i) / rho
// prod_{j != i} (lambda_j - d_i) / (d_j - d_i)|) (Gu-Eisenstat; each factor
// is O(1) by interlacing).
__global__ void __launch_bounds__(256) k_dc_zhat(const DcNode *__restrict__ nodes,
                                                 const int2 *__restrict__ wmap, int nw, int n,
                                                 DcArrays ar) {
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (q >= nw) return;
  const int2 wm = wmap[q];
  const DcNode nd = nodes[wm.x];
  const int off = nd.off, i = wm.y;
  if (i == nd.s - 1) {
    // the node's deflation rotations, in order, on its Qp columns (each lane
    // keeps its rows, so the wavefront's program order orders them)
    const int nr = ar.nrot[off];
    for (int e = 0; e < nr; ++e) {
      double *x = ar.Qp + off + (int64_t)n * (off + ar.rot_x[off + e]);
      double *y = ar.Qp + off + (int64_t)n * (off + ar.rot_y[off + e]);
      const double c = ar.rot_c[off + e], sn = ar.rot_s[off + e];
      for (int r = lane; r < nd.s; r += 64) {
        const double a = x[r], b = y[r];
        x[r] = c * a + sn * b;
        y[r] = c * b - sn * a;
      }
    }
  }
  const double *__restrict__ dd = ar.dd;
  const double *__restrict__ zz = ar.zz;
  const double *__restrict__ dels = ar.dels;
  const double *rho_in = ar.rho;
  double *__restrict__ zh = ar.zh;
  const int k = ar.kk[off];
  if (i >= k) return;
  const double di = dd[off + i];
  double p = 1.0;
  for (int j = lane; j < k; j += 64) {
    const double dl = dels[(off + i) + (int64_t)n * (off + j)];   // d_i - lambda_j
    p *= (j == i) ? -dl / rho_in[off] : -dl / (dd[off + j] - di);
  }
#pragma unroll
  for (int msk = 32; msk > 0; msk >>= 1) p *= __shfl_xor(p, msk);
  if (lane == 0) zh[off + i] = copysign(sqrt(fabs(p)), zz[off + i]);
}

// One wavefront per (node, Qp column j): the rank of its eigenvalue among
// the node's s (the k roots dv[0..k), the deflated values dv[k..s); ties by
// column) gives lam[off + rank] and csrc[off + rank] = j; for a root, column
// j of U, u_i = zh_i / (d_i - lambda_j), normalised.
__global__ void __launch_bounds__(256) k_dc_ucol(const DcNode *__restrict__ nodes,
                                                 const int2 *__restrict__ wmap, int nw, int n,
                                                 DcArrays ar) {
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (q >= nw) return;
  const int2 wm = wmap[q];
  const DcNode nd = nodes[wm.x];
  const int off = nd.off, j = wm.y;
  const double x = ar.dv[off + j];
  double below = 0.0;
  for (int t = lane; t < nd.s; t += 64) {
    const double y = ar.dv[off + t];
    below += ((y < x) || (y == x && t < j)) ? 1.0 : 0.0;
  }
  const int rank = (int)wave_sum_all(below);
  if (lane == 0) {
    ar.lam[off + rank] = x;
    ar.csrc[off + rank] = j;
  }
  const int k = ar.kk[off];
  if (j >= k) return;
  const double *__restrict__ zh = ar.zh;
  const double *__restrict__ dels = ar.dels;
  double *__restrict__ U = ar.U;
  double u[kKR];
  double um = 0.0;
#pragma unroll
  for (int r = 0; r < kKR; ++r) {
    const int i = lane + 64 * r;
    u[r] = i < k ? zh[off + i] / dels[(off + i) + (int64_t)n * (off + j)] : 0.0;
    um = fmax(um, fabs(u[r]));
  }
  // normalised with the entries scaled by the largest one (no underflow of
  // the squares when the entries are tiny, no overflow when they are huge)
  const double sc = 1.0 / wave_max_all(um);
  double ss = 0.0;
#pragma unroll
  for (int r = 0; r < kKR; ++r) ss = fma(u[r] * sc, u[r] * sc, ss);
  const double inv = sc / sqrt(wave_sum_all(ss));
#pragma unroll
  for (int r = 0; r < kKR; ++r) {
    const int i = lane + 64 * r;
    if (i < k) U[(off + i) + (int64_t)n * (off + j)] = u[r] * inv;
  }
}

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One wavefront per 16 x 16 output tile (node, tile row, tile column) of the
// node's new eigenvectors: output column c takes Qp column t = csrc[c]; for
// t < k (a root) it is Qp[:, 0..k) U[:, t] (FP64 matrix cores; lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16], result register r is
// D[l / 16 + 4 r][l % 16]), otherwise the deflated column Qp[:, t] itself.
__global__ void __launch_bounds__(256) k_dc_gemm(const DcNode *__restrict__ nodes,
                                                 const int4 *__restrict__ tiles, int nt, int n,
                                                 const int *__restrict__ kk,
                                                 const int *__restrict__ csrc,
                                                 const double *__restrict__ Qp,
                                                 const double *__restrict__ U,
                                                 double *__restrict__ Qc) {
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (q >= nt) return;
  const int4 tl = tiles[q];
  const DcNode nd = nodes[tl.x];
  const int off = nd.off, s = nd.s;
  const int k = kk[off];
  const int lr = l & 15, lk = l >> 4;
  const int arow = 16 * tl.y + lr;            // A operand row
  const int bcol = 16 * tl.z + lr;            // B operand (output) column
  const int tb = bcol < s ? csrc[off + bcol] : k;
  const bool arow_in = arow < s, broot = tb < k;
  const double *Ap = Qp + (off + arow) + (int64_t)n * off;
  const double *Bp = U + off + (int64_t)n * (off + (broot ? tb : 0));
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  int u0 = 0;
  for (; u0 + 16 <= k; u0 += 16) {
    double a[4], b[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int u = u0 + 4 * h + lk;
      a[h] = arow_in ? Ap[(int64_t)n * u] : 0.0;
      b[h] = broot ? Bp[u] : 0.0;
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) acc = mfma_f64(a[h], b[h], acc);
  }
  for (; u0 < k; u0 += 4) {
    const int u = u0 + lk;
    const double a = (arow_in && u < k) ? Ap[(int64_t)n * u] : 0.0;
    const double b = (broot && u < k) ? Bp[u] : 0.0;
    acc = mfma_f64(a, b, acc);
  }
  const int c = 16 * tl.z + lr;
  if (c >= s) return;
  const int t = csrc[off + c];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * tl.y + lk + 4 * r;
    if (row < s) {
      const int64_t o = (off + row) + (int64_t)n * (off + c);
      Qc[o] = t < k ? acc[r] : Qp[(off + row) + (int64_t)n * (off + t)];
    }
  }
}

// Back-transformation: x = H_0 H_1 ... H_{n-3} z (reflectors applied last to
// first), written to W[:, n - 1 - c] with w[n - 1 - c] = lam[c] (descending
// order).  One workgroup of 4 wavefronts per 4 eigenvectors, one each in
// registers (lane l: rows l + 64 m, m < RM); 4 rather than 8 per workgroup
// puts twice as many CUs to work (15 % faster at n = 480).  Reflectors come
// in chunks of 16 staged in LDS (rows padded to 64 RM); the next chunk's
// loads are in flight while the current one is applied.
constexpr int kBackVecs = 4;
template <int RM>
__global__ void __launch_bounds__(64 * kBackVecs) k_dc_back(int n, const double *__restrict__ hv,
                                                const double *__restrict__ htau,
                                                const double *__restrict__ Qc,
                                                const double *__restrict__ lam,
                                                double *__restrict__ w, double *__restrict__ W,
                                                int64_t ldw) {
  constexpr int NT = 64 * kBackVecs, NP = 64 * RM, CH = 16, U = CH * NP / NT;
  __shared__ double vs[CH * NP];
  __shared__ double ts[CH];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int c = blockIdx.x * kBackVecs + wv;
  const bool has = c < n;
  double z[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const int i = lane + 64 * m;
    z[m] = (has && i < n) ? Qc[i + (int64_t)n * c] : 0.0;
  }
  // chunk with highest reflector k1 holds k1 - 15 .. k1 (those >= 0)
  double nx[U], nt = 0.0;
  auto load = [&](int k1) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + NT * u, r = e / NP, i = e % NP;
      const int k = k1 - (CH - 1) + r;
      nx[u] = (k >= 0 && i < n) ? hv[(int64_t)k * n + i] : 0.0;
    }
    const int k = k1 - (CH - 1) + tid;
    nt = (tid < CH && k >= 0) ? htau[k] : 0.0;
  };
  if (n >= 3) load(n - 3);
  for (int k1 = n - 3; k1 >= 0; k1 -= CH) {
    __syncthreads();   // the previous chunk has been applied
#pragma unroll
    for (int u = 0; u < U; ++u) vs[tid + NT * u] = nx[u];
    if (tid < CH) ts[tid] = nt;
    __syncthreads();
    if (k1 - CH >= 0) load(k1 - CH);
    // reflectors k1, k1 - 1, ..., k1 - 15 (slot r = CH - 1 .. 0; absent ones
    // have tau = 0)
    for (int r = CH - 1; r >= 0; --r) {
      const double *v = vs + r * NP;
      double sm = 0.0;
#pragma unroll
      for (int m = 0; m < RM; ++m) sm = fma(v[lane + 64 * m], z[m], sm);
      sm = ts[r] * wave_sum_all(sm);
#pragma unroll
      for (int m = 0; m < RM; ++m) z[m] = fma(-sm, v[lane + 64 * m], z[m]);
    }
  }
  if (!has) return;
  const int oc = n - 1 - c;
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const int i = lane + 64 * m;
    if (i < n) W[i + ldw * oc] = z[m];
  }
  if (lane == 0) w[oc] = lam[c];
}

__global__ void k_latch_fail(const int *fail, int *err) {
  if (*fail != 0 && *err == 0) *err = FKF_E_HIP;
}

__global__ void k_zero_d(double *p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

__global__ void k_zero_ints(int *p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

}  // namespace

bool sym_eig_dc_supported(int n) { return n >= 3 && n <= kDcMaxN; }

// Host driver: merge tree and launch tables are built once per order n.
void sym_eig_dc(const double *A, int64_t lda, int n, double *w, double *W, int64_t ldw,
                hipStream_t st, EigWork &ws, int *err) {
  FKF_REQUIRE(sym_eig_dc_supported(n), "sym_eig_dc: order out of range");
  if (ws.dc_n != n) {
    // merges of the halving tree, grouped by height (children first)
    std::vector<std::vector<DcNode>> by_h;
    auto rec = [&](auto &&self, int off, int s) -> int {
      if (s == 1) return 0;
      const int m = s / 2;
      const int h = 1 + std::max(self(self, off, m), self(self, off + m, s - m));
      if ((int)by_h.size() < h) by_h.resize(h);
      by_h[h - 1].push_back(DcNode{off, s, m, 0});
      return h;
    };
    rec(rec, 0, n);
    // raw tables: nodes (off, s, m, 0), waves (node, i), tiles (node, row, col, 0)
    std::vector<int32_t> raw, wraw, traw;
    ws.dc_levels.clear();
    for (const auto &lv : by_h) {
      EigWork::DcLevel L;
      L.node0 = (int)(raw.size() / 4);
      L.nodes = (int)lv.size();
      L.wave0 = (int)(wraw.size() / 2);
      L.tile0 = (int)(traw.size() / 4);
      for (const DcNode &d : lv) {
        const int idx = (int)(raw.size() / 4);
        raw.insert(raw.end(), {d.off, d.s, d.m, 0});
        for (int i = 0; i < d.s; ++i) wraw.insert(wraw.end(), {idx, i});
        const int nt = (d.s + 15) / 16;
        for (int a = 0; a < nt; ++a)
          for (int b = 0; b < nt; ++b) traw.insert(traw.end(), {idx, a, b, 0});
      }
      L.waves = (int)(wraw.size() / 2) - L.wave0;
      L.tiles = (int)(traw.size() / 4) - L.tile0;
      ws.dc_levels.push_back(L);
    }
    ws.dc_nodes.upload(raw, st);
    ws.dc_wmap.upload(wraw, st);
    ws.dc_tiles.upload(traw, st);
    FKF_CHECK_HIP(hipStreamSynchronize(st));   // host temporaries
    ws.dc_n = n;
  }
  const size_t nn = (size_t)n * n;
  ws.hv.reserve(nn);
  ws.Qc.reserve(nn);
  ws.Qp.reserve(nn);
  ws.U.reserve(nn);
  ws.dels.reserve(nn);
  ws.vec.reserve((size_t)19 * n);
  ws.ivec.reserve((size_t)6 * n + 2);
  double *htau = ws.vec.p, *dg = htau + n, *eg = dg + n, *xb = eg + n;   // xb: 8n words
  DcArrays ar;
  ar.lam = xb + 8 * n;
  ar.dd = ar.lam + n;
  ar.zz = ar.dd + n;
  ar.dv = ar.zz + n;
  ar.zh = ar.dv + n;
  ar.rho = ar.zh + n;
  ar.rot_c = ar.rho + n;
  ar.rot_s = ar.rot_c + n;
  ar.Qc = ws.Qc.p;
  ar.Qp = ws.Qp.p;
  ar.U = ws.U.p;
  ar.dels = ws.dels.p;
  ar.kk = ws.ivec.p;
  ar.csrc = ar.kk + n;
  ar.qsrc = ar.csrc + n;
  ar.rot_x = ar.qsrc + n;
  ar.rot_y = ar.rot_x + n;
  ar.nrot = ar.rot_y + n;
  int *sync = ar.nrot + n;
  double *lam = ar.lam;
  {
    FKF_TRACE("eig_tridiag", st);
    // columns in registers: RM rows per lane (n <= 64 RM), at most 8 CW
    // columns per workgroup; for 256 < n <= 512 one column per wavefront (60
    // workgroups at n = 480: 6 % faster than two columns per wavefront on
    // 30); at most 64 workgroups for every order, so that four reductions on
    // separate streams always fit the chip together
    // exchange words (tags 0) and the failure flag cleared by kernels
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, sync, 1);
    hipLaunchKernelGGL(k_zero_d, dim3((unsigned)((8 * n + 255) / 256)), dim3(256), 0, st, xb,
                       8 * n);
    auto launch = [&](auto kern, int cmax) {
      const int G = (n + cmax - 1) / cmax;
      hipLaunchKernelGGL(kern, dim3(G), dim3(kTrThreads), 0, st, A, lda, n, G, ws.hv.p, htau, dg,
                         eg, reinterpret_cast<unsigned long long *>(xb), sync);
    };
    if (n <= 128)
      launch(k_tridiag<2, 8>, 64);
    else if (n <= 256)
      launch(k_tridiag<4, 8>, 64);
    else if (n <= 512)
      launch(k_tridiag<8, 1>, 8);
    else
      launch(k_tridiag<16, 2>, 16);
  }
  {
    FKF_TRACE("eig_dc", st);
    hipLaunchKernelGGL(k_dc_leaves, dim3((n + 255) / 256), dim3(256), 0, st, dg, eg, n, lam,
                       ws.Qc.p);
    const DcNode *nodes = reinterpret_cast<const DcNode *>(ws.dc_nodes.p);
    const int2 *wmap = reinterpret_cast<const int2 *>(ws.dc_wmap.p);
    const int4 *tiles = reinterpret_cast<const int4 *>(ws.dc_tiles.p);
    for (const auto &L : ws.dc_levels) {
      const DcNode *nl = nodes + L.node0;
      // wave and tile tables index nodes globally
      hipLaunchKernelGGL(k_dc_prep, dim3(L.nodes), dim3(kPrepThreads), 0, st, nl, n, eg, ar);
      const unsigned gw = (unsigned)((L.waves + 3) / 4);
      hipLaunchKernelGGL(k_dc_secular, dim3(gw), dim3(256), 0, st, nodes, wmap + L.wave0, L.waves,
                         n, ar);
      hipLaunchKernelGGL(k_dc_zhat, dim3(gw), dim3(256), 0, st, nodes, wmap + L.wave0, L.waves, n,
                         ar);
      hipLaunchKernelGGL(k_dc_ucol, dim3(gw), dim3(256), 0, st, nodes, wmap + L.wave0, L.waves, n,
                         ar);
      hipLaunchKernelGGL(k_dc_gemm, dim3((unsigned)((L.tiles + 3) / 4)), dim3(256), 0, st, nodes,
                         tiles + L.tile0, L.tiles, n, ar.kk, ar.csrc, ws.Qp.p, ws.U.p, ws.Qc.p);
    }
  }
  {
    FKF_TRACE("eig_back", st);
    auto back = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3((unsigned)((n + kBackVecs - 1) / kBackVecs)),
                         dim3(64 * kBackVecs), 0, st, n, ws.hv.p, htau,
                         ws.Qc.p, lam, w, W, ldw);
    };
    if (n <= 128)
      back(k_dc_back<2>);
    else if (n <= 256)
      back(k_dc_back<4>);
    else if (n <= 512)
      back(k_dc_back<8>);
    else
      back(k_dc_back<16>);
  }
  FKF_CHECK_HIP(hipGetLastError());
  // a failed exchange (workgroups that never met) is reported, not hidden
  if (err) {
    hipLaunchKernelGGL(k_latch_fail, dim3(1), dim3(1), 0, st, sync, err);
    FKF_CHECK_HIP(hipGetLastError());
    return;
  }
  if (!ws.cnt_host) FKF_CHECK_HIP(hipHostMalloc((void **)&ws.cnt_host, 4 * sizeof(int)));
  FKF_CHECK_HIP(hipMemcpyAsync(ws.cnt_host + 3, sync, sizeof(int), hipMemcpyDeviceToHost, st));
  FKF_CHECK_HIP(hipStreamSynchronize(st));
  if (ws.cnt_host[3] != 0)
    throw Error{FKF_E_HIP, "sym_eig_dc: the reduction's workgroups did not all run together"};
}

}  // namespace fkf
