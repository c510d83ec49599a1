// Dense and sparse FP64 linear algebra on the GPU for the filter's data-space
// quantities: the measurement operator products, the n_m x n_m innovation
// Gram matrix and its eigen-decomposition (the projected eigenproblem of the
// generalized eigenvalue problem, Section 2.2.2), and tall GEMMs.
#include <algorithm>
#include <vector>

#include "kernels.h"
#include "linalg.h"
#include "trace.h"

namespace fkf {

// ===================================================== block Jacobi eigen ===
// Cyclic two-sided Jacobi in a block-parallel order.  The padded matrix
// (np = multiple of 32) is split into nb = np/16 blocks of 16 indices.  A
// round pairs the blocks by a round-robin tournament; in each pair's 32 x 32
// principal submatrix (in LDS) the rotations of the round are applied,
// giving an orthogonal J_k, and then every 32 x 32 tile of A is updated as
// J_k1^T A J_k2 and V as V J_k.  A sweep (nb - 1 rounds) rotates every index
// pair once; the iteration stops when the off-diagonal Frobenius norm falls
// below tol ||A||_F (1e-12 unless the caller asks otherwise; or a sweep
// rotates nothing).  Padding indices carry
// zero rows/columns and are never rotated.

constexpr int kJB = 16;   // block size
constexpr int kJT = 32;   // tile (pair) size

__device__ __forceinline__ int rr_player(int pos, int round, int m) {
  return pos == 0 ? 0 : 1 + ((pos - 1 + round) % (m - 1));
}

__device__ __forceinline__ int pair_index(int k, int i, int round, int nb) {
  int P = rr_player(k, round, nb), Q = rr_player(nb - 1 - k, round, nb);
  return i < kJB ? P * kJB + i : Q * kJB + (i - kJB);
}

// Rotation (c, s) for the 2 x 2 symmetric block [app apq; apq aqq]: with
// zeta = aqq - app and eta = 2 apq, t = sign(zeta) eta / (|zeta| + sqrt(zeta^2
// + eta^2)) is the smaller root of t^2 + 2 tau t - 1 = 0 (tau = zeta / eta).
// The angle is evaluated on (zeta, eta) scaled to [-1, 1] with the hardware
// FP64 reciprocal and reciprocal square root (no refinement: a short
// dependency chain, accurate to far more than the next sweep needs); c = 1 /
// sqrt(1 + t^2) (hardware seed y0, e = 1 - q y0^2, then one third-order step
// y0 (1 + e/2 + 3 e^2/8)) and s = t c make the applied rotation orthogonal to
// FP64 rounding, so the entry apq is reduced by the angle's relative error
// rather than zeroed, and the next sweep removes the remainder.  Branch-free;
// skipped (identity) when |apq| <= max(tol_rel sqrt|app aqq|, tol_abs)
// (compared in squares).
__device__ __forceinline__ bool jacobi_rotation(double app, double aqq, double apq, double tol_rel,
                                                double tol_abs, double &c, double &s) {
  const double a2 = apq * apq;
  const bool rot = a2 > tol_rel * tol_rel * fabs(app * aqq) && a2 > tol_abs * tol_abs;
  const double z = aqq - app, e = 2.0 * apq;
  const double sc = __builtin_amdgcn_rcp(rot ? fmax(fabs(z), fabs(e)) : 1.0);
  const double zs = z * sc, es = e * sc;
  const double h2 = fma(zs, zs, es * es);   // in [1, 2] when rot
  const double den = fabs(zs) + h2 * __builtin_amdgcn_rsq(rot ? h2 : 1.0);
  const double t = (zs < 0.0 ? -es : es) * __builtin_amdgcn_rcp(den);
  const double q = fma(t, t, 1.0);
  const double y0 = __builtin_amdgcn_rsq(q);
  const double ey = fma(-q * y0, y0, 1.0);
  const double y = fma(y0 * ey, fma(0.375, ey, 0.5), y0);
  c = rot ? y : 1.0;
  s = rot ? t * y : 0.0;
  return rot;
}

// Batched form: blockIdx.y (or .z) selects problem b; problem b's padded
// matrices start at b * np * np, its rotations at b * npair * 32 * 32, its
// norms at b * (2 + np) (fro[0] = ||A||_F, fro[1] = relative off-diagonal
// norm, fro[2..] column partials) and its counters at b * (3 + np)
// (cnt[0] = workgroups that rotated in the sweep, cnt[1..np] rank scratch,
// cnt[1 + np] = convergence flag, cnt[2 + np] = A buffer holding the
// converged matrix, or -1).
__global__ void k_jacobi_init(const EigProblem *__restrict__ pr, int np, double *__restrict__ Ap,
                              double *__restrict__ V) {
  const int b = blockIdx.y;
  const EigProblem q = pr[b];
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)np * np) return;
  int i = (int)(e % np), j = (int)(e / np);
  const int64_t o = (int64_t)b * np * np;
  Ap[o + e] = (i < q.n && j < q.n) ? q.A[i + q.lda * j] : 0.0;
  V[o + e] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_set_int(int *p, int v) { *p = v; }

// cnt[b * stride] = v for every problem b
__global__ void k_set_int_strided(int *p, int64_t stride, int count, int v) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < count) p[b * stride] = v;
}

// Convergence flags after a sweep: problem b has converged when its relative
// off-diagonal norm is <= tol or none of its workgroups rotated anything (a
// converged problem stays converged).  done_host[0] = 1 when all have.
__global__ void k_eig_converged(const double *__restrict__ fro, int *__restrict__ cnt, int np,
                                int count, double tol, int cur_buf, int *__restrict__ done_host) {
  __shared__ int all;
  if (threadIdx.x == 0) all = 1;
  __syncthreads();
  for (int b = threadIdx.x; b < count; b += blockDim.x) {
    const double *f = fro + (int64_t)b * (2 + np);
    int *c = cnt + (int64_t)b * (3 + np);
    const int was = c[1 + np];
    const int d = (was != 0 || f[1] <= tol || c[0] == 0) ? 1 : 0;
    if (d && !was) c[2 + np] = cur_buf;   // later launches leave this problem's A there
    c[1 + np] = d;
    if (!d) all = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) done_host[0] = all;
}

// Off-diagonal sum of squares: one workgroup per (column, problem)
// (partials), then one workgroup per problem sums them in a fixed order.
__global__ void __launch_bounds__(256) k_offnorm_cols(const double *__restrict__ A, int np,
                                                      double *__restrict__ fro, int with_diag) {
  __shared__ double red[4];
  const int j = blockIdx.x, b = blockIdx.y;
  const double *Ab = A + (int64_t)b * np * np;
  double s = 0;
  for (int i = threadIdx.x; i < np; i += 256) {
    double v = Ab[i + (int64_t)np * j];
    if (i != j || with_diag) s = fma(v, v, s);
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) fro[(int64_t)b * (2 + np) + 2 + j] = red[0] + red[1] + red[2] + red[3];
}

// initial: fro[0] = sqrt(sum); else fro[1] = sqrt(sum) / fro[0]
__global__ void __launch_bounds__(256) k_offnorm_final(double *__restrict__ fro, int np,
                                                       int initial) {
  __shared__ double red[4];
  double *f = fro + (int64_t)blockIdx.x * (2 + np);
  double s = 0;
  for (int j = threadIdx.x; j < np; j += 256) s += f[2 + j];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0] + red[1] + red[2] + red[3];
    if (initial)
      f[0] = sqrt(t);
    else
      f[1] = f[0] > 0 ? sqrt(t) / f[0] : 0.0;
  }
}

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Position of block B in the pairing of round r: pair index k and half h
// (0: first block of the pair, 1: second).  Inverse of rr_player.
__device__ __forceinline__ void block_slot(int B, int r, int nb, int &k, int &h) {
  if (B == 0) {
    k = 0;
    h = 0;
    return;
  }
  const int m = nb - 1;
  const int pos = ((B - 1 - r) % m + m) % m + 1;
  if (pos < nb / 2) {
    k = pos;
    h = 0;
  } else {
    k = nb - 1 - pos;
    h = 1;
  }
}

// Rotations of one round on the 32 x 32 principal submatrix of block pair k
// (local indices 0..15: block P, 16..31: block Q).  Every index pair (i, j)
// of the matrix is rotated exactly once per sweep, so a sweep is one cyclic
// Jacobi sweep in a block-parallel order: the round visits the 256 cross
// pairs (i in P, j in Q) in 16 sub-rounds of 16 disjoint rotations (i with
// 16 + (i + u) mod 16), and the first round of a sweep also visits the pairs
// within each block beforehand (15 sub-rounds, round-robin within P and Q).
// intra_pair: the pair of index k of a within-block sub-round u (k < 8: the
// 8 pairs of block P, k >= 8: those of block Q).
__device__ __forceinline__ void intra_pair(int u, int k, int &p, int &q) {
  const int base = k < kJB / 2 ? 0 : kJB, kk = k & (kJB / 2 - 1);
  p = base + rr_player(kk, u, kJB);
  q = base + rr_player(kJB - 1 - kk, u, kJB);
}

constexpr int kTS = kJT * (kJT + 1);   // doubles in one padded 32 x 32 LDS tile
// LDS of a round: solve part = 2 tiles + J (rotation phase), or 4 products
// M (32 x 16) over tiles 1-2, 4 tiles of A and 2 halves of J' (formation);
// update part = 4 tiles
constexpr int kRoundSmem = 7 * kTS + 2 * kJT * 17;

// Solve part of a round (one workgroup per block pair k of round r).  The
// pair's tile is either read from A (no rotations pending) or formed from the
// previous round's state: with the previous round's rotations J' pending,
// block (X, Y) of the tile is J'_X^T A'[X', Y'] J'_Y, where X' is the previous
// pair tile holding block X and J'_X its 16 columns for X; each wave forms one
// of the four 16 x 16 blocks on the FP64 matrix cores.  Then the rotations of
// the round: the tile is double-buffered in LDS; in a sub-round every thread
// reads the current tile, computes the two rotations of its 2 x 2 pair block
// itself (branch-free) and writes its four entries of the next tile; rows of
// J = prod R are updated in place; one barrier per sub-round.
__device__ void jacobi_solve_part(double *smem, const double *__restrict__ A, int np, int nb,
                                  const int32_t *__restrict__ pidx, int k, int r, int rprev,
                                  const double *__restrict__ Jprev,
                                  const double *__restrict__ fro, double *__restrict__ Jout,
                                  int *cnt) {
  // pidx[(round * npair + pair) * 32 + i]: global index of local index i
  const int npair = nb / 2;
  const int32_t *ix = pidx + ((int64_t)r * npair + k) * kJT;
  double(*S0)[kJT + 1] = reinterpret_cast<double(*)[kJT + 1]>(smem);
  double(*S1)[kJT + 1] = reinterpret_cast<double(*)[kJT + 1]>(smem + kTS);
  double(*Jm)[kJT + 1] = reinterpret_cast<double(*)[kJT + 1]>(smem + 2 * kTS);
  __shared__ int rot_any;
  const int tid = threadIdx.x;
  if (rprev < 0) {
    for (int e = tid; e < kJT * kJT; e += 256) {
      int i = e & 31, j = e >> 5;
      S0[i][j] = A[ix[i] + (int64_t)np * ix[j]];
    }
  } else {
    // regions: M (4 x 32 x 16) over S1 and Jm; T (4 tiles) and the J' halves after them
    double *Mb = smem + kTS;
    double *Tb = smem + 3 * kTS;
    double *Jh = smem + 7 * kTS;   // [2][32][17]
    const int wv = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    const int blk[2] = {rr_player(k, r, nb), rr_player(nb - 1 - k, r, nb)};
    int kp[2], hp[2];
    block_slot(blk[0], rprev, nb, kp[0], hp[0]);
    block_slot(blk[1], rprev, nb, kp[1], hp[1]);
    // wave wv: block (X, Y) = (wv >> 1, wv & 1); its previous tile (kp[X], kp[Y])
    const int X = wv >> 1, Y = wv & 1;
    double *T = Tb + wv * kTS;
    {
      // all global loads of the formation first (J' halves and the previous
      // tile, indices computed rather than looked up), then the LDS stores,
      // so that the loads share one memory latency
      double jv[2 * kJT * kJB / 256];
#pragma unroll
      for (int it = 0; it < 2 * kJT * kJB / 256; ++it) {
        const int e = tid + 256 * it;
        const int x = e / (kJT * kJB), a = (e >> 4) & 31, c = e & 15;
        jv[it] = Jprev[(int64_t)kp[x] * kJT * kJT + a + kJT * (hp[x] * kJB + c)];
      }
      const int gi = pair_index(kp[X], l & 31, rprev, nb);
      double v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q)
        v[q] = A[gi + (int64_t)np * pair_index(kp[Y], (l >> 5) + 2 * q, rprev, nb)];
#pragma unroll
      for (int it = 0; it < 2 * kJT * kJB / 256; ++it) {
        const int e = tid + 256 * it;
        const int x = e / (kJT * kJB), a = (e >> 4) & 31, c = e & 15;
        Jh[(x * kJT + a) * 17 + c] = jv[it];
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) T[(l & 31) * (kJT + 1) + (l >> 5) + 2 * q] = v[q];
    }
    __syncthreads();
    // M (32 x 16) = T (32 x 32) J'_Y (32 x 16)
    double *M = Mb + wv * (kJT * kJB);
    const double *JY = Jh + Y * kJT * 17, *JX = Jh + X * kJT * 17;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) {
      v4d acc = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
        acc = mfma_f64(T[(16 * ti + lr) * (kJT + 1) + 4 * kk + lk], JY[(4 * kk + lk) * 17 + lr],
                       acc);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) M[(16 * ti + lk + 4 * rr) * kJB + lr] = acc[rr];
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's LDS writes are done
    __builtin_amdgcn_wave_barrier();
    // block (16 x 16) = J'_X^T (16 x 32) M (32 x 16)
    v4d acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
      acc = mfma_f64(JX[(4 * kk + lk) * 17 + lr], M[(4 * kk + lk) * kJB + lr], acc);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) S0[kJB * X + lk + 4 * rr][kJB * Y + lr] = acc[rr];
    __syncthreads();
  }
  for (int e = tid; e < kJT * kJT; e += 256) {
    int i = e & 31, j = e >> 5;
    Jm[i][j] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) rot_any = 0;
  const double tol_abs = 1e-15 * fro[0], tol_rel = 1e-15;
  const int P1 = tid >> 4, P2 = tid & 15;
  const int jr = tid >> 4;   // J rows jr and jr + 16, column pair P2
  double(*Sc)[kJT + 1] = S0;
  double(*Sn)[kJT + 1] = S1;
  // One sub-round: this thread's 2 x 2 block (rows p1, q1; columns p2, q2)
  // of the next tile and its entries of J (rows jr, jr + 16; columns p2, q2).
  // The J entries are read with the tile entries, before the rotations, so
  // that both reads share one LDS latency.  Each thread computes the rotation
  // of its column pair P2 only: its row pair P1 (< 16) is the column pair of
  // lane P1 of the same wavefront, whose rotation is read across lanes.
  auto sub_round = [&](int p1, int q1, int p2, int q2) {
    const double a21 = Sc[p2][p2], a22 = Sc[q2][q2], a23 = Sc[p2][q2];
    const double b11 = Sc[p1][p2], b12 = Sc[p1][q2];
    const double b21 = Sc[q1][p2], b22 = Sc[q1][q2];
    const double jp0 = Jm[jr][p2], jq0 = Jm[jr][q2];
    const double jp1 = Jm[jr + 16][p2], jq1 = Jm[jr + 16][q2];
    double c2, s2;
    const bool r2 = jacobi_rotation(a21, a22, a23, tol_rel, tol_abs, c2, s2);
    if (r2 && P1 == 0) rot_any = 1;
    const double c1 = __shfl(c2, P1), s1 = __shfl(s2, P1);
    const double t11 = c2 * b11 - s2 * b12, t12 = s2 * b11 + c2 * b12;
    const double t21 = c2 * b21 - s2 * b22, t22 = s2 * b21 + c2 * b22;
    Sn[p1][p2] = c1 * t11 - s1 * t21;
    Sn[p1][q2] = c1 * t12 - s1 * t22;
    Sn[q1][p2] = s1 * t11 + c1 * t21;
    Sn[q1][q2] = s1 * t12 + c1 * t22;
    Jm[jr][p2] = c2 * jp0 - s2 * jq0;
    Jm[jr][q2] = s2 * jp0 + c2 * jq0;
    Jm[jr + 16][p2] = c2 * jp1 - s2 * jq1;
    Jm[jr + 16][q2] = s2 * jp1 + c2 * jq1;
    double(*t)[kJT + 1] = Sc;
    Sc = Sn;
    Sn = t;
    __syncthreads();
  };
  __syncthreads();
  if (r == 0) {
    // first round of a sweep: the pairs within each block (round-robin)
    for (int u = 0; u < kJB - 1; ++u) {
      int p1, q1, p2, q2;
      intra_pair(u, P1, p1, q1);
      intra_pair(u, P2, p2, q2);
      sub_round(p1, q1, p2, q2);
    }
  }
#pragma unroll
  for (int u = 0; u < kJB; ++u)
    sub_round(P1, kJB + ((P1 + u) & (kJB - 1)), P2, kJB + ((P2 + u) & (kJB - 1)));
  double *Jo = Jout + (int64_t)k * kJT * kJT;
  for (int e = tid; e < kJT * kJT; e += 256) {
    int i = e & 31, j = e >> 5;
    Jo[i + kJT * j] = Jm[i][j];
  }
  if (tid == 0 && rot_any) atomicAdd(cnt, 1);
}

// Update part of a round (one workgroup per output tile): with the round's
// rotations J (pairs of round r), every 32 x 32 tile of A (rows of pair k1,
// columns of pair k2) becomes J_k1^T A J_k2 (read from Acur, written to
// Anext) and every 32-row tile of V becomes V J_k2 (in place).  Both products
// run on the FP64 matrix cores, one 16 x 16 output quarter per wavefront
// (v_mfma_f64_16x16x4f64: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
// result register r is D[l / 16 + 4 r][l % 16]).
__device__ void jacobi_update_part(double *smem, int w, const double *__restrict__ Acur,
                                   double *__restrict__ Anext, double *__restrict__ V, int np,
                                   int nb, const int32_t *__restrict__ pidx, int r,
                                   const double *__restrict__ Jbuf) {
  double(*Tl)[kJT + 1] = reinterpret_cast<double(*)[kJT + 1]>(smem);
  double(*J1)[kJT + 1] = reinterpret_cast<double(*)[kJT + 1]>(smem + kTS);
  double(*J2)[kJT + 1] = reinterpret_cast<double(*)[kJT + 1]>(smem + 2 * kTS);
  double(*Tm)[kJT + 1] = reinterpret_cast<double(*)[kJT + 1]>(smem + 3 * kTS);
  const int npair = nb / 2;
  const int tilesA = npair * npair;
  const int tid = threadIdx.x;
  const bool isA = w < tilesA;
  int k1, k2, rc0 = 0;
  if (isA) {
    k1 = w / npair;
    k2 = w % npair;
  } else {
    w -= tilesA;
    rc0 = (w / npair) * kJT;
    k1 = -1;
    k2 = w % npair;
  }
  // global indices of the pairs' local indices, computed (round-robin
  // tournament) rather than looked up, so that the data loads do not wait on
  // index loads
  const int gi1 = isA ? pair_index(k1, tid & 31, r, nb) : 0;
  {
    double tv[kJT * kJT / 256], j1v[kJT * kJT / 256], j2v[kJT * kJT / 256];
#pragma unroll
    for (int it = 0; it < kJT * kJT / 256; ++it) {
      const int e = tid + 256 * it;
      const int i = e & 31, j = e >> 5;
      const int gj = pair_index(k2, j, r, nb);
      if (isA) {
        tv[it] = Acur[gi1 + (int64_t)np * gj];
        j1v[it] = Jbuf[(int64_t)k1 * kJT * kJT + i + kJT * j];
      } else {
        tv[it] = V[rc0 + i + (int64_t)np * gj];
      }
      j2v[it] = Jbuf[(int64_t)k2 * kJT * kJT + i + kJT * j];
    }
#pragma unroll
    for (int it = 0; it < kJT * kJT / 256; ++it) {
      const int e = tid + 256 * it;
      const int i = e & 31, j = e >> 5;
      Tl[i][j] = tv[it];
      if (isA) J1[i][j] = j1v[it];
      J2[i][j] = j2v[it];
    }
  }
  __syncthreads();
  const int wv = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
  const int ti = wv >> 1, tj = wv & 1;   // this wave's 16 x 16 output quarter
  v4d acc = {0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < 8; ++kk)
    acc = mfma_f64(Tl[16 * ti + lr][4 * kk + lk], J2[4 * kk + lk][16 * tj + lr], acc);
  if (!isA) {
    const int gj = pair_index(k2, 16 * tj + lr, r, nb);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * ti + lk + 4 * q;
      V[rc0 + i + (int64_t)np * gj] = acc[q];
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) Tm[16 * ti + lk + 4 * q][16 * tj + lr] = acc[q];
  __syncthreads();
  acc = v4d{0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < 8; ++kk)
    acc = mfma_f64(J1[4 * kk + lk][16 * ti + lr], Tm[4 * kk + lk][16 * tj + lr], acc);
  const int gj = pair_index(k2, 16 * tj + lr, r, nb);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 16 * ti + lk + 4 * q;
    Anext[pair_index(k1, i, r, nb) + (int64_t)np * gj] = acc[q];
  }
}

// One launch per round for every problem of the batch (blockIdx.y):
// workgroups [0, npair) solve the pairs of round r (when solve_on), the rest
// apply the pending rotations of round rprev (when rprev >= 0) to A
// (Acur -> Anext) and V.  The two parts only read Acur, so they run
// concurrently; one LDS region serves either part.  A problem that has
// converged skips the launch entirely.
__global__ void __launch_bounds__(256) k_jacobi_round(const double *__restrict__ Acur,
                                                      double *__restrict__ Anext,
                                                      double *__restrict__ V, int np, int nb,
                                                      const int32_t *__restrict__ pidx,
                                                      int r, int solve_on, int rprev,
                                                      const double *__restrict__ Jprev,
                                                      double *__restrict__ Jcur,
                                                      const double *__restrict__ fro, int *cnt) {
  __shared__ double smem[kRoundSmem];
  const int b = blockIdx.y;
  int *c = cnt + (int64_t)b * (3 + np);
  if (c[1 + np]) return;   // converged: this problem's part of the launch is empty
  const int npair = nb / 2;
  const int64_t oa = (int64_t)b * np * np, oj = (int64_t)b * npair * kJT * kJT;
  const int nsolve = solve_on ? npair : 0;
  if ((int)blockIdx.x < nsolve)
    jacobi_solve_part(smem, Acur + oa, np, nb, pidx, blockIdx.x, r, rprev, Jprev + oj,
                      fro + (int64_t)b * (2 + np), Jcur + oj, c);
  else
    jacobi_update_part(smem, blockIdx.x - nsolve, Acur + oa, Anext + oa, V + oa, np, nb, pidx,
                       rprev, Jprev + oj);
}

// Eigenvalues from the diagonal, ranked in descending order (ties by index),
// one workgroup per problem.
__global__ void __launch_bounds__(1024) k_eig_rank(const EigProblem *__restrict__ pr,
                                                   const double *__restrict__ A0,
                                                   const double *__restrict__ A1, int last_buf,
                                                   int np, int *__restrict__ cnt) {
  const int b = blockIdx.x;
  const EigProblem q = pr[b];
  int *c = cnt + (int64_t)b * (3 + np);
  const int buf = c[2 + np] >= 0 ? c[2 + np] : last_buf;
  const double *Ap = (buf ? A1 : A0) + (int64_t)b * np * np;
  int *rank = c + 1;
  for (int i = threadIdx.x; i < q.n; i += 1024) {
    double li = Ap[i + (int64_t)np * i];
    int r = 0;
    for (int j = 0; j < q.n; ++j) {
      double lj = Ap[j + (int64_t)np * j];
      r += (lj > li) || (lj == li && j < i);
    }
    q.w[r] = li;
    rank[i] = r;
  }
}

__global__ void k_eig_vecs(const EigProblem *__restrict__ pr, const double *__restrict__ V, int np,
                           const int *__restrict__ cnt) {
  const int b = blockIdx.z;
  const EigProblem q = pr[b];
  int r = blockIdx.y * blockDim.x + threadIdx.x;
  int i = blockIdx.x;
  if (i >= q.n || r >= q.n) return;
  const int *rank = cnt + (int64_t)b * (3 + np) + 1;
  q.W[r + q.ldw * rank[i]] = V[(int64_t)b * np * np + r + (int64_t)np * i];
}

EigWork::~EigWork() {
  if (cnt_host) (void)hipHostFree(cnt_host);
  if (ev) (void)hipEventDestroy(ev);
}

int sym_eig_batched(const EigProblem *probs, int count, hipStream_t st, EigWork &ws, double tol,
                    int *err) {
  if (count == 1 && sym_eig_dc_supported(probs[0].n)) {
    const EigProblem &p = probs[0];
    sym_eig_dc(p.A, p.lda, p.n, p.w, p.W, p.ldw, st, ws, err);
    return 0;
  }
  int nmax = 0;
  for (int b = 0; b < count; ++b) nmax = std::max(nmax, probs[b].n);
  if (count <= 0 || nmax <= 0) return 0;
  const int np = (nmax + kJT - 1) / kJT * kJT;
  const int nb = np / kJB;
  const int npair = nb / 2;
  const size_t sq = (size_t)np * np * count;
  ws.A.reserve(sq);
  ws.A2.reserve(sq);
  ws.V.reserve(sq);
  ws.J.reserve((size_t)npair * kJT * kJT * count);
  ws.J2.reserve((size_t)npair * kJT * kJT * count);
  ws.fro.reserve((size_t)(2 + np) * count);
  ws.cnt.reserve((size_t)(3 + np) * count);
  if (!ws.cnt_host) FKF_CHECK_HIP(hipHostMalloc((void **)&ws.cnt_host, 4 * sizeof(int)));
  if (!ws.ev) FKF_CHECK_HIP(hipEventCreateWithFlags(&ws.ev, hipEventDisableTiming));
  if (ws.pidx_np != np) {
    // global index of local index i of pair k in round r (round-robin tournament)
    std::vector<int32_t> t((size_t)(nb - 1) * npair * kJT);
    auto player = [&](int pos, int r) { return pos == 0 ? 0 : 1 + ((pos - 1 + r) % (nb - 1)); };
    for (int r = 0; r < nb - 1; ++r)
      for (int k = 0; k < npair; ++k)
        for (int i = 0; i < kJT; ++i) {
          const int P = player(k, r), Q = player(nb - 1 - k, r);
          t[((size_t)r * npair + k) * kJT + i] = i < kJB ? P * kJB + i : Q * kJB + (i - kJB);
        }
    ws.pidx.upload(t, st);
    FKF_CHECK_HIP(hipStreamSynchronize(st));   // t is a host temporary
    ws.pidx_np = np;
  }
  std::vector<EigProblem> hp(probs, probs + count);
  ws.probs.upload(hp, st);
  FKF_CHECK_HIP(hipStreamSynchronize(st));     // hp is a host temporary
  const int64_t cstride = 3 + np;
  int64_t tot = (int64_t)np * np;
  hipLaunchKernelGGL(k_jacobi_init, dim3((unsigned)((tot + 255) / 256), count), dim3(256), 0, st,
                     ws.probs.p, np, ws.A.p, ws.V.p);
  hipLaunchKernelGGL(k_offnorm_cols, dim3(np, count), dim3(256), 0, st, ws.A.p, np, ws.fro.p, 1);
  hipLaunchKernelGGL(k_offnorm_final, dim3(count), dim3(256), 0, st, ws.fro.p, np, 1);
  hipLaunchKernelGGL(k_set_int_strided, dim3((count + 255) / 256), dim3(256), 0, st,
                     ws.cnt.p + 1 + np, cstride, count, 0);
  hipLaunchKernelGGL(k_set_int_strided, dim3((count + 255) / 256), dim3(256), 0, st,
                     ws.cnt.p + 2 + np, cstride, count, -1);
  const unsigned grid_upd = (unsigned)(npair * npair + (np / kJT) * npair);
  // Rounds are launched as k_jacobi_round: the solve of round r runs next to
  // the update of round r - 1 (A double-buffered, J double-buffered); the last
  // update of a sweep runs alone before the convergence test.  A problem has
  // converged when its relative off-diagonal norm is below tol (a
  // perturbation of at most tol ||A||_F on the eigenvalues) or a sweep
  // rotates nothing; the batch stops when all have.  The test of sweep s is
  // read on the host while sweep s + 1 is already queued (no idle GPU during
  // the host round trip); launches of a converged problem are empty.
  double *Ab[2] = {ws.A.p, ws.A2.p};
  double *Jb[2] = {ws.J.p, ws.J2.p};
  int ca = 0, cj = 0;   // current A buffer; J buffer written by the next solve
  volatile int *done_host = ws.cnt_host + 2;
  int sweeps = 0, ca_prev = 0;
  for (int sw = 0; sw < 40; ++sw) {
    hipLaunchKernelGGL(k_set_int_strided, dim3((count + 255) / 256), dim3(256), 0, st, ws.cnt.p,
                       cstride, count, 0);
    int rprev = -1;
    {
      // the sweep's nb launches are timed as one interval (no events between
      // the back-to-back round kernels)
      FKF_TRACE_N("eig_jacobi_round", st, nb);
      for (int r = 0; r <= nb - 1; ++r) {
        const bool solve = r < nb - 1;
        const unsigned grid = (solve ? npair : 0) + (rprev >= 0 ? grid_upd : 0);
        hipLaunchKernelGGL(k_jacobi_round, dim3(grid, count), dim3(256), 0, st, Ab[ca],
                           Ab[ca ^ 1], ws.V.p, np, nb, ws.pidx.p, r, solve ? 1 : 0, rprev,
                           Jb[cj ^ 1], Jb[cj], ws.fro.p, ws.cnt.p);
        if (rprev >= 0) ca ^= 1;   // the update wrote the other A buffer
        if (solve) {
          cj ^= 1;                 // this solve's rotations are pending now
          rprev = r;
        }
      }
    }
    hipLaunchKernelGGL(k_offnorm_cols, dim3(np, count), dim3(256), 0, st, Ab[ca], np, ws.fro.p, 0);
    hipLaunchKernelGGL(k_offnorm_final, dim3(count), dim3(256), 0, st, ws.fro.p, np, 0);
    // wait for the previous sweep's flags (this sweep is queued behind them)
    if (sw > 0) {
      FKF_CHECK_HIP(hipEventSynchronize(ws.ev));
      if (*done_host) {
        ca = ca_prev;   // this sweep's launches were empty
        break;
      }
    }
    ++sweeps;
    *done_host = 0;
    hipLaunchKernelGGL(k_eig_converged, dim3(1), dim3(256), 0, st, ws.fro.p, ws.cnt.p, np, count,
                       tol, ca, (int *)done_host);
    FKF_CHECK_HIP(hipEventRecord(ws.ev, st));
    ca_prev = ca;
    if (sw == 39) FKF_CHECK_HIP(hipEventSynchronize(ws.ev));
  }
  hipLaunchKernelGGL(k_eig_rank, dim3(count), dim3(1024), 0, st, ws.probs.p, Ab[0], Ab[1], ca, np,
                     ws.cnt.p);
  hipLaunchKernelGGL(k_eig_vecs, dim3(np, (unsigned)((np + 255) / 256), count), dim3(256), 0, st,
                     ws.probs.p, ws.V.p, np, ws.cnt.p);
  FKF_CHECK_HIP(hipGetLastError());
  return sweeps;
}

int sym_eig(const double *A, int64_t lda, int n, double *w, double *W, int64_t ldw,
            hipStream_t st, EigWork &ws, double tol, int *err) {
  if (n <= 0) return 0;
  if (sym_eig_dc_supported(n)) {
    sym_eig_dc(A, lda, n, w, W, ldw, st, ws, err);
    return 0;
  }
  EigProblem p{A, lda, n, 0, w, W, ldw};
  return sym_eig_batched(&p, 1, st, ws, tol);
}

}  // namespace fkf

extern "C" fkf_status fkf_sym_eig(const double *A, int64_t lda, int32_t n, double *w,
                                  double *W, int64_t ldw, void *stream) {
  using namespace fkf;
  return guarded([&] {
    FKF_REQUIRE(n >= 1, "fkf_sym_eig: n must be positive");
    FKF_REQUIRE(lda >= n && ldw >= n, "fkf_sym_eig: leading dimensions must be >= n");
    FKF_REQUIRE(A && w && W, "fkf_sym_eig: null pointer");
    hipStream_t st = as_stream(stream);
    EigWork ws;
    sym_eig(A, lda, n, w, W, ldw, st, ws, 1e-12, nullptr);
    FKF_CHECK_HIP(hipGetLastError());
    FKF_CHECK_HIP(hipStreamSynchronize(st));   // ws is freed on return
  });
}

namespace fkf {

// ========================================================= sparse products ===
__global__ void __launch_bounds__(256) k_spmv(const int64_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ col,
                                              const double *__restrict__ val, int n_m,
                                              const double *__restrict__ x, double *__restrict__ y) {
  int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= n_m) return;
  int l = threadIdx.x & 63;
  double s = 0;
  for (int64_t e = rowptr[m] + l; e < rowptr[m + 1]; e += 64) s = fma(val[e], x[col[e]], s);
  s = wave_sum(s);
  if (l == 0) y[m] = s;
}

void spmv(const int64_t *rowptr, const int32_t *col, const double *val, int n_m, const double *x,
          double *y, hipStream_t st) {
  if (n_m <= 0) return;
  hipLaunchKernelGGL(k_spmv, dim3((n_m + 3) / 4), dim3(256), 0, st, rowptr, col, val, n_m, x, y);
}

__global__ void k_fill(double *__restrict__ p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void fill(double *p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

__global__ void __launch_bounds__(64) k_scatter_ht(const int64_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ col,
                                                   const double *__restrict__ val, int64_t n,
                                                   double *__restrict__ D) {
  int m = blockIdx.x;
  for (int64_t e = rowptr[m] + threadIdx.x; e < rowptr[m + 1]; e += 64)
    D[col[e] + n * m] = val[e];
}

void dense_ht(const int64_t *rowptr, const int32_t *col, const double *val, int n_m, int64_t n,
              double *D, hipStream_t st) {
  fill(D, n * n_m, 0.0, st);
  if (n_m > 0)
    hipLaunchKernelGGL(k_scatter_ht, dim3(n_m), dim3(64), 0, st, rowptr, col, val, n, D);
}

// G = H P (n_m x n_m) for CSR H and P (n x n_m, ld n), upper triangle: one
// wavefront per (row m of H, 8 columns of P that reach the diagonal or beyond,
// j0 + 7 >= m); lanes run over the row's entries (cells in index order, so
// neighbouring lanes mostly read neighbouring rows of P) and each entry is
// read once for the eight columns.  Entries left of the diagonal in a group
// that straddles it are formed too but not read.
constexpr int kGramCols = 8;
__global__ void __launch_bounds__(256) k_gram_hp(const int64_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col,
                                                 const double *__restrict__ val, int n_m, int64_t n,
                                                 const double *__restrict__ P,
                                                 double *__restrict__ G) {
  const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ngrp = (n_m + kGramCols - 1) / kGramCols;
  if (wv >= (int64_t)n_m * ngrp) return;
  const int m = (int)(wv % n_m), j0 = (int)(wv / n_m) * kGramCols;
  if (j0 + kGramCols - 1 < m) return;   // group left of the diagonal
  const int l = threadIdx.x & 63;
  double s[kGramCols];
#pragma unroll
  for (int u = 0; u < kGramCols; ++u) s[u] = 0.0;
  for (int64_t q = rowptr[m] + l; q < rowptr[m + 1]; q += 64) {
    const double v = val[q];
    const double *Pc = P + col[q];
#pragma unroll
    for (int u = 0; u < kGramCols; ++u)
      if (j0 + u < n_m) s[u] = fma(v, Pc[n * (j0 + u)], s[u]);
  }
#pragma unroll
  for (int u = 0; u < kGramCols; ++u) {
    const double t = wave_sum_all(s[u]);
    if (l == 0 && j0 + u < n_m) G[m + (int64_t)n_m * (j0 + u)] = t;
  }
}
// H Gamma H^T is symmetric: the upper triangle of G as formed defines it.
// The lower triangle of G is filled from the upper one (threads below the
// diagonal read only entries above it, which no thread writes), and
// A = R^-1/2 G R^-1/2.
__global__ void k_gram_sym(double *__restrict__ G, int n_m, const double *__restrict__ r,
                           double *__restrict__ A) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n_m * n_m) return;
  int m = (int)(e % n_m), j = (int)(e / n_m);
  double g;
  if (j >= m) {
    g = G[e];
  } else {
    g = G[j + (int64_t)n_m * m];
    G[e] = g;
  }
  A[e] = g / sqrt(r[m] * r[j]);
}

void innovation_gram(const int64_t *rowptr, const int32_t *col, const double *val, int n_m,
                     int64_t n, const double *P, const double *noise_var, double *G, double *A,
                     hipStream_t st) {
  int64_t e = (int64_t)n_m * n_m;
  if (e == 0) return;
  const int64_t waves = (int64_t)n_m * ((n_m + kGramCols - 1) / kGramCols);
  hipLaunchKernelGGL(k_gram_hp, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, rowptr, col,
                     val, n_m, n, P, G);
  hipLaunchKernelGGL(k_gram_sym, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, G, n_m,
                     noise_var, A);
}

// ==================================================================== GEMM ===
// C = A B, 64 x 64 output tile per workgroup, 4 x 4 per thread, k in chunks of 16.
__global__ void __launch_bounds__(256) k_gemm_nn(int64_t m, int n, int k, const double *__restrict__ A,
                                                 int64_t lda, const double *__restrict__ B,
                                                 int64_t ldb, double *__restrict__ C, int64_t ldc) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * 64;
  const int n0 = blockIdx.y * 64;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int k0 = 0; k0 < k; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = tid + 256 * q;
      int r = e & 63, kk = e >> 6;
      int64_t gr = m0 + r;
      int gk = k0 + kk;
      As[kk][r] = (gr < m && gk < k) ? A[gr + lda * gk] : 0.0;
      int kb = e & 15, c = e >> 4;
      int gkb = k0 + kb, gc = n0 + c;
      Bs[kb][c] = (gkb < k && gc < n) ? B[gkb + ldb * gc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int64_t gr = m0 + tx + 16 * a;
      int gc = n0 + ty + 16 * b;
      if (gr < m && gc < n) C[gr + ldc * gc] = acc[a][b];
    }
}

static bool tall_shape(int64_t m, int64_t n, int64_t k);
static void gemm_tall(int64_t m, int n, int k, double alpha, const double *A, int64_t lda,
                      const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                      hipStream_t st);

void gemm_nn(int64_t m, int n, int k, const double *A, int64_t lda, const double *B, int64_t ldb,
             double *C, int64_t ldc, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  if (tall_shape(m, n, k)) {
    gemm_tall(m, n, k, 1.0, A, lda, B, ldb, 0.0, C, ldc, st);
    return;
  }
  hipLaunchKernelGGL(k_gemm_nn, dim3((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64)),
                     dim3(256), 0, st, m, n, k, A, lda, B, ldb, C, ldc);
}

__global__ void k_scale_rows(int64_t m, int n, const double *__restrict__ s, double *__restrict__ A,
                             int64_t lda) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  int64_t i = e % m, j = e / m;
  A[i + lda * j] *= s[i];
}

void scale_rows(int64_t m, int n, const double *s, double *A, int64_t lda, hipStream_t st) {
  int64_t e = m * n;
  if (e <= 0) return;
  hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, m, n, s, A,
                     lda);
}

}  // namespace fkf

namespace fkf {

// ============================================================ general GEMM ===
// C = alpha op(A) op(B) + beta C (FP64, column-major), 64 x 64 output tiles,
// 4 x 4 per thread, k in chunks of 16.  With split > 1 the k range is divided
// among grid.z slices whose partial products go to a workspace and are summed
// in slice order by k_gemm_combine (deterministic).
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm_gen(int64_t m, int64_t n, int64_t k, double alpha,
                                                  const double *__restrict__ A, int64_t lda,
                                                  const double *__restrict__ B, int64_t ldb,
                                                  double beta, double *__restrict__ C, int64_t ldc,
                                                  int64_t kslice, double *__restrict__ part) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * 64, n0 = (int64_t)blockIdx.y * 64;
  const int64_t kb = (int64_t)blockIdx.z * kslice, ke = min(k, kb + kslice);
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int64_t k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = tid + 256 * q;
      // A tile: As[kk][r] = op(A)[m0 + r][k0 + kk]
      {
        int r, kk;
        if (!TA) { r = e & 63; kk = e >> 6; } else { kk = e & 15; r = e >> 4; }
        int64_t gr = m0 + r, gk = k0 + kk;
        double v = 0.0;
        if (gr < m && gk < ke) v = TA ? A[gk + lda * gr] : A[gr + lda * gk];
        As[kk][r] = v;
      }
      // B tile: Bs[kk][c] = op(B)[k0 + kk][n0 + c]
      {
        int c, kk;
        if (!TB) { kk = e & 15; c = e >> 4; } else { c = e & 63; kk = e >> 6; }
        int64_t gk = k0 + kk, gc = n0 + c;
        double v = 0.0;
        if (gc < n && gk < ke) v = TB ? B[gc + ldb * gk] : B[gk + ldb * gc];
        Bs[kk][c] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int64_t gr = m0 + tx + 16 * a, gc = n0 + ty + 16 * b;
      if (gr < m && gc < n) {
        if (part) {
          part[(int64_t)blockIdx.z * m * n + gr + m * gc] = acc[a][b];
        } else {
          double v = alpha * acc[a][b];
          if (beta != 0.0) v += beta * C[gr + ldc * gc];
          C[gr + ldc * gc] = v;
        }
      }
    }
}

__global__ void k_gemm_combine(int64_t m, int64_t n, int splits, double alpha,
                               const double *__restrict__ part, double beta,
                               double *__restrict__ C, int64_t ldc) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  int64_t i = e % m, j = e / m;
  double s = 0;
  for (int z = 0; z < splits; ++z) s += part[(int64_t)z * m * n + e];
  double v = alpha * s;
  if (beta != 0.0) v += beta * C[i + ldc * j];
  C[i + ldc * j] = v;
}

// C = alpha A B + beta C for a tall A (m x k, m large) and a short B (k x n),
// column-major, on the FP64 matrix cores: one workgroup of eight wavefronts
// per 64 rows x 256 columns, two workgroups per CU (10 % faster than 512
// columns per workgroup, one per CU).  Per 16-entry chunk of k the 64 x 16
// block of A goes through LDS (double-buffered, one barrier per chunk; loaded
// one chunk ahead, coalesced down the columns); wavefront w multiplies it with
// columns [32 w, 32 w + 32) of B, whose operands it reads from global memory one chunk
// ahead (four consecutive k of a column share a 32-byte sector).  Rows past
// m and k past the end are zero in LDS; column blocks past n are skipped.
__global__ void __launch_bounds__(512, 2) k_gemm_tall(int64_t m, int n, int k, double alpha,
                                                   const double *__restrict__ A, int64_t lda,
                                                   const double *__restrict__ B, int64_t ldb,
                                                   double beta, double *__restrict__ C,
                                                   int64_t ldc) {
  constexpr int LDK = 18;
  __shared__ double As[2][64 * LDK];
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int lr = l & 15, lk = l >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * 64;
  const int rows = (int)min((int64_t)64, m - m0);
  const int nrb = (rows + 15) >> 4;
  const int c0 = blockIdx.y * 256 + 32 * w;
  const int ncb = min(2, max(0, (n - c0 + 15) >> 4));
  const int ar = tid & 63, ak = 2 * (tid >> 6);   // A staging: row ar, chunk columns ak, ak + 1
  auto load_a = [&](int k0, double *a2) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kk = k0 + ak + h;
      a2[h] = (ar < rows && kk < k) ? A[m0 + ar + lda * (int64_t)kk] : 0.0;
    }
  };
  auto load_b = [&](int k0, double *b) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int kb = k0 + 4 * kk + lk;
      const int kc = kb < k ? kb : 0;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int cc = c0 + 16 * j + lr;
        b[2 * kk + j] = B[kc + ldb * (int64_t)(cc < n ? cc : 0)];
      }
    }
  };
  v4d acc[4][2];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[q][j] = v4d{0, 0, 0, 0};
  double anext[2], bcur[8], bnext[8];
  load_a(0, anext);
  load_b(0, bcur);
  int buf = 0;
  for (int k0 = 0; k0 < k; k0 += 16) {
    As[buf][ar * LDK + ak] = anext[0];
    As[buf][ar * LDK + ak + 1] = anext[1];
    if (k0 + 16 < k) {
      load_a(k0 + 16, anext);
      load_b(k0 + 16, bnext);
    }
    __syncthreads();
    const double *As_ = As[buf];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < nrb) {
          const double a = As_[(16 * q + lr) * LDK + 4 * kk + lk];
#pragma unroll
          for (int j = 0; j < 2; ++j)
            if (j < ncb) acc[q][j] = mfma_f64(a, bcur[2 * kk + j], acc[q][j]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) bcur[i] = bnext[i];
    buf ^= 1;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * q + lk + 4 * r;
        const int cc = c0 + 16 * j + lr;
        if (i < rows && cc < n) {
          double *c = C + m0 + i + ldc * (int64_t)cc;
          *c = beta != 0.0 ? fma(alpha, acc[q][j][r], beta * *c) : alpha * acc[q][j][r];
        }
      }
}

static bool tall_shape(int64_t m, int64_t n, int64_t k) {
  return m >= 4096 && n >= 1 && n <= INT32_MAX && k >= 1 && k <= INT32_MAX;
}

static void gemm_tall(int64_t m, int n, int k, double alpha, const double *A, int64_t lda,
                      const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_gemm_tall, dim3((unsigned)((m + 63) / 64), (unsigned)((n + 255) / 256)),
                     dim3(512), 0, st, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

void gemm(bool ta, bool tb, int64_t m, int64_t n, int64_t k, double alpha, const double *A,
          int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
          hipStream_t st, DevBuf<double> *work) {
  if (m <= 0 || n <= 0) return;
  if (k <= 0) {
    // C = beta C
    if (beta == 0.0) {
      for (int64_t j = 0; j < n; ++j) fill(C + ldc * j, m, 0.0, st);
    } else if (beta != 1.0) {
      throw Error{FKF_E_UNSUPPORTED, "gemm: k = 0 with beta not in {0, 1}"};
    }
    return;
  }
  if (!ta && !tb && tall_shape(m, n, k)) {
    gemm_tall(m, (int)n, (int)k, alpha, A, lda, B, ldb, beta, C, ldc, st);
    return;
  }
  const int64_t tm = (m + 63) / 64, tn = (n + 63) / 64;
  int splits = 1;
  if (work && tm * tn < 1024 && k >= 1024) {
    // long reductions with a small output (W^T U and the like): enough
    // k-slices for about 2048 workgroups
    splits = (int)std::min<int64_t>((2048 + tm * tn - 1) / (tm * tn), k / 256);
    splits = std::max(splits, 1);
  }
  int64_t kslice = (k + splits - 1) / splits;
  kslice = (kslice + 15) / 16 * 16;
  splits = (int)((k + kslice - 1) / kslice);
  double *part = nullptr;
  if (splits > 1) {
    work->reserve((size_t)splits * m * n);
    part = work->p;
  }
  dim3 grid((unsigned)tm, (unsigned)tn, (unsigned)splits);
  auto kern = ta ? (tb ? k_gemm_gen<true, true> : k_gemm_gen<true, false>)
                 : (tb ? k_gemm_gen<false, true> : k_gemm_gen<false, false>);
  hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                     kslice, part);
  if (splits > 1)
    hipLaunchKernelGGL(k_gemm_combine, dim3((unsigned)((m * n + 255) / 256)), dim3(256), 0, st, m,
                       n, splits, alpha, part, beta, C, ldc);
}

// ========================================================= sparse x dense ===
// out (n_m x cols, ld n_m) = H X for CSR H and X (n x cols, ld ldx).
__global__ void __launch_bounds__(256) k_sp_dense(const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col,
                                                  const double *__restrict__ val, int n_m,
                                                  const double *__restrict__ X, int64_t ldx,
                                                  int cols, double *__restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= (int64_t)n_m * cols) return;
  int m = (int)(e % n_m), j = (int)(e / n_m);
  int l = threadIdx.x & 63;
  const double *Xj = X + ldx * j;
  double s = 0;
  for (int64_t q = rowptr[m] + l; q < rowptr[m + 1]; q += 64) s = fma(val[q], Xj[col[q]], s);
  s = wave_sum(s);
  if (l == 0) out[m + (int64_t)n_m * j] = s;
}

void sp_dense(const int64_t *rowptr, const int32_t *col, const double *val, int n_m,
              const double *X, int64_t ldx, int cols, double *out, hipStream_t st) {
  int64_t e = (int64_t)n_m * cols;
  if (e <= 0) return;
  hipLaunchKernelGGL(k_sp_dense, dim3((unsigned)((e + 3) / 4)), dim3(256), 0, st, rowptr, col, val,
                     n_m, X, ldx, cols, out);
}

// ======================================================== Cholesky solve ===
// S (m x m, ld m) = L L^T in place (lower triangle), then x = S^-1 b
// overwriting b.  Blocked right-looking factorization over panels of
// kCholNB columns: one launch factors the panel's diagonal block, one solves
// the block column below it, the plain GEMM updates the trailing matrix, and
// one workgroup finally runs the two triangular solves.  A non-positive (or
// non-finite) pivot is recorded in *flag; the solve then sets
// *err = FKF_E_NOT_SPD and leaves b unchanged.
constexpr int kCholNB = 32;

// Panel p, diagonal block: one wavefront factors the nb x nb block (already
// updated by the panels to its left) in LDS, lane l owning row l, writes L_pp
// back (lower triangle) and records a bad pivot in *flag.
__global__ void __launch_bounds__(64) k_chol_diag(double *__restrict__ S, int m, int p,
                                                  int *__restrict__ flag) {
  __shared__ double D[kCholNB][kCholNB + 1];
  const int l = threadIdx.x;
  const int nb = min(kCholNB, m - p);
  if (l < nb)
    for (int c = 0; c <= l; ++c) D[l][c] = S[(p + l) + (int64_t)m * (p + c)];
  __syncthreads();
  int bad = 0;
  for (int j = 0; j < nb; ++j) {
    const double d = D[j][j];
    const bool ok = d > 0.0 && isfinite(d);
    bad |= !ok;
    const double piv = ok ? sqrt(d) : 1.0;
    __syncthreads();
    if (l == j) D[j][j] = piv;
    if (l > j && l < nb) D[l][j] /= piv;
    __syncthreads();
    if (l > j && l < nb) {
      const double lj = D[l][j];
      for (int c = j + 1; c <= l; ++c) D[l][c] -= lj * D[c][j];
    }
    __syncthreads();
  }
  if (l < nb)
    for (int c = 0; c <= l; ++c) S[(p + l) + (int64_t)m * (p + c)] = D[l][c];
  if (l == 0) {
    if (p == 0) *flag = bad;
    else if (bad) *flag = 1;
  }
}

// Panel p, block column: X L_pp^T = A for the rows below the diagonal block,
// one row per lane, 64 rows per workgroup (L_pp read from S after
// k_chol_diag has written it).
__global__ void __launch_bounds__(64) k_chol_panel(double *__restrict__ S, int m, int p) {
  __shared__ double D[kCholNB][kCholNB + 1];
  const int l = threadIdx.x;
  const int nb = min(kCholNB, m - p);
  if (l < nb)
    for (int c = 0; c <= l; ++c) D[l][c] = S[(p + l) + (int64_t)m * (p + c)];
  __syncthreads();
  const int i = p + nb + 64 * blockIdx.x + l;
  if (i >= m) return;
  double x[kCholNB];
#pragma unroll
  for (int c = 0; c < kCholNB; ++c) x[c] = c < nb ? S[i + (int64_t)m * (p + c)] : 0.0;
#pragma unroll
  for (int c = 0; c < kCholNB; ++c) {
    if (c < nb) {
      double v = x[c];
#pragma unroll
      for (int q = 0; q < c; ++q) v -= x[q] * D[c][q];
      x[c] = v / D[c][c];
    }
  }
#pragma unroll
  for (int c = 0; c < kCholNB; ++c)
    if (c < nb) S[i + (int64_t)m * (p + c)] = x[c];
}

// Forward (L y = b) and backward (L^T x = y) substitution by one workgroup,
// panel by panel: wavefront 0 solves the nb x nb triangle with lane l owning
// entry l; the other rows are updated by the whole workgroup (forward: row
// updates, coalesced down the panel's columns; backward: one wavefront-wide
// dot product per panel column).
__global__ void __launch_bounds__(1024) k_chol_trsv(const double *__restrict__ S, int m,
                                                    double *__restrict__ b,
                                                    const int *__restrict__ flag, int *err,
                                                    double *__restrict__ ll_acc) {
  __shared__ double xs[kCholNB];
  __shared__ double red[2][16];
  if (*flag) {
    if (threadIdx.x == 0) atomicExch(err, (int)FKF_E_NOT_SPD);
    return;
  }
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  for (int p = 0; p < m; p += kCholNB) {
    const int nb = min(kCholNB, m - p);
    if (w == 0) {
      double v = l < nb ? b[p + l] : 0.0;
      const double dg = l < nb ? S[(p + l) + (int64_t)m * (p + l)] : 1.0;
      for (int c = 0; c < nb; ++c) {
        const double xc = __shfl(v / dg, c);
        if (l == c) v = xc;
        else if (l > c && l < nb) v -= S[(p + l) + (int64_t)m * (p + c)] * xc;
      }
      if (l < nb) {
        xs[l] = v;
        b[p + l] = v;
      }
    }
    __syncthreads();
    for (int i = p + nb + tid; i < m; i += 1024) {
      double acc = b[i];
      for (int c = 0; c < nb; ++c) acc -= S[i + (int64_t)m * (p + c)] * xs[c];
      b[i] = acc;
    }
    __syncthreads();
  }
  if (ll_acc) {
    // Gaussian log-density of b: with y = L^-1 b (now in b),
    // -(y^T y + 2 sum log L_ii + m log 2 pi) / 2
    double q = 0.0, ld = 0.0;
    for (int i = tid; i < m; i += 1024) {
      q = fma(b[i], b[i], q);
      ld += log(S[i + (int64_t)m * i]);
    }
    q = wave_sum(q);
    ld = wave_sum(ld);
    if (l == 0) {
      red[0][w] = q;
      red[1][w] = ld;
    }
    __syncthreads();
    if (tid == 0) {
      double qs = 0.0, ls = 0.0;
      for (int v = 0; v < 16; ++v) {
        qs += red[0][v];
        ls += red[1][v];
      }
      ll_acc[0] += -0.5 * (qs + 2.0 * ls + (double)m * log(2.0 * M_PI));
    }
    __syncthreads();
  }
  const int last = (m - 1) / kCholNB * kCholNB;
  for (int p = last; p >= 0; p -= kCholNB) {
    const int nb = min(kCholNB, m - p);
    for (int c = w; c < nb; c += 16) {
      double acc = 0.0;
      for (int i = p + nb + l; i < m; i += 64) acc = fma(S[i + (int64_t)m * (p + c)], b[i], acc);
      acc = wave_sum(acc);
      if (l == 0) xs[c] = b[p + c] - acc;
    }
    __syncthreads();
    if (w == 0) {
      double v = l < nb ? xs[l] : 0.0;
      const double dg = l < nb ? S[(p + l) + (int64_t)m * (p + l)] : 1.0;
      for (int c = nb - 1; c >= 0; --c) {
        const double xc = __shfl(v / dg, c);
        if (l == c) v = xc;
        else if (l < c) v -= S[(p + c) + (int64_t)m * (p + l)] * xc;
      }
      if (l < nb) b[p + l] = v;
    }
    __syncthreads();
  }
}

void chol_solve(double *S, int m, double *b, int *flag, int *err, hipStream_t st,
                double *ll_acc) {
  if (m <= 0) return;
  for (int p = 0; p < m; p += kCholNB) {
    const int nb = std::min(kCholNB, m - p);
    const int below = m - p - nb;
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(64), 0, st, S, m, p, flag);
    if (below > 0) {
      hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)((below + 63) / 64)), dim3(64), 0, st, S, m,
                         p);
      double *L21 = S + (p + nb) + (int64_t)m * p;
      double *A22 = S + (p + nb) + (int64_t)m * (p + nb);
      gemm(false, true, below, below, nb, -1.0, L21, m, L21, m, 1.0, A22, m, st, nullptr);
    }
  }
  hipLaunchKernelGGL(k_chol_trsv, dim3(1), dim3(1024), 0, st, S, m, b, flag, err, ll_acc);
}

// Scale column j of a column-major m x n matrix by s[j] (in place).
__global__ void k_scale_cols(int64_t m, int n, const double *__restrict__ s, double *__restrict__ A,
                             int64_t lda) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  int64_t i = e % m, j = e / m;
  A[i + lda * j] *= s[j];
}

void scale_cols(int64_t m, int n, const double *s, double *A, int64_t lda, hipStream_t st) {
  int64_t e = m * n;
  if (e <= 0) return;
  hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, m, n, s, A,
                     lda);
}

__global__ void k_scale2d(int64_t m, int n, double a, double *__restrict__ A, int64_t lda) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  A[e % m + lda * (e / m)] *= a;
}

void scale2d(int64_t m, int n, double a, double *A, int64_t lda, hipStream_t st) {
  int64_t e = m * n;
  if (e <= 0) return;
  hipLaunchKernelGGL(k_scale2d, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, m, n, a, A, lda);
}

// A = (A + A^T) / 2 for a square m x m matrix (ld m).
__global__ void k_symmetrize(double *__restrict__ A, int m) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  int i = (int)(e % m), j = (int)(e / m);
  if (i < j) {
    double v = 0.5 * (A[i + (int64_t)m * j] + A[j + (int64_t)m * i]);
    A[i + (int64_t)m * j] = v;
    A[j + (int64_t)m * i] = v;
  }
}

void symmetrize(double *A, int m, hipStream_t st) {
  int64_t e = (int64_t)m * m;
  if (e <= 0) return;
  hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, A, m);
}

// Copy a column-major m x n block (lda) to (ldb).
__global__ void k_copy2d(int64_t m, int n, const double *__restrict__ A, int64_t lda,
                         double *__restrict__ B, int64_t ldb) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  int64_t i = e % m, j = e / m;
  B[i + ldb * j] = A[i + lda * j];
}

void copy2d(int64_t m, int n, const double *A, int64_t lda, double *B, int64_t ldb, hipStream_t st) {
  int64_t e = m * n;
  if (e <= 0) return;
  hipLaunchKernelGGL(k_copy2d, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, m, n, A, lda, B,
                     ldb);
}

}  // namespace fkf
