// Dense and sparse FP64 linear algebra on the GPU for the filter's data-space
// quantities: the measurement operator products, the n_m x n_m innovation
// Gram matrix and its eigen-decomposition (the projected eigenproblem of the
// generalized eigenvalue problem, Section 2.2.2), and tall GEMMs.
#include <algorithm>

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
// below 1e-12 ||A||_F (or a sweep rotates nothing).  Padding indices carry
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

// Rotation (c, s) that annihilates apq in the 2 x 2 symmetric block
// [app apq; apq aqq]: with zeta = aqq - app and eta = 2 apq,
// t = sign(zeta) eta / (|zeta| + sqrt(zeta^2 + eta^2)) is the smaller root of
// t^2 + 2 tau t - 1 = 0 (tau = zeta / eta), c = 1 / sqrt(1 + t^2), s = t c.
// Branch-free (the skip test selects the identity), so two rotations of one
// thread are evaluated as independent instruction streams.  Skipped when
// |apq| <= max(tol_rel sqrt|app aqq|, tol_abs) (compared in squares).
__device__ __forceinline__ bool jacobi_rotation(double app, double aqq, double apq, double tol_rel,
                                                double tol_abs, double &c, double &s) {
  const double a2 = apq * apq;
  const bool rot = a2 > tol_rel * tol_rel * fabs(app * aqq) && a2 > tol_abs * tol_abs;
  const double zeta = aqq - app, eta = 2.0 * apq;
  const double q = fma(zeta, zeta, eta * eta);
  const double r = q * rsq_nr(rot ? q : 1.0);
  const double t = copysign(1.0, zeta) * eta * rcp_nr(rot ? fabs(zeta) + r : 1.0);
  const double cc = rsq_nr(fma(t, t, 1.0));
  c = rot ? cc : 1.0;
  s = rot ? t * cc : 0.0;
  return rot;
}

__global__ void k_jacobi_init(const double *__restrict__ A, int64_t lda, int n, int np,
                              double *__restrict__ Ap, double *__restrict__ V) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)np * np) return;
  int i = (int)(e % np), j = (int)(e / np);
  Ap[e] = (i < n && j < n) ? A[i + lda * j] : 0.0;
  V[e] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_set_int(int *p, int v) { *p = v; }

// Off-diagonal sum of squares: one workgroup per column (partials), then
// off[0] = sqrt(sum of partials) / fro in a fixed order.
__global__ void __launch_bounds__(256) k_offnorm_cols(const double *__restrict__ A, int np,
                                                      double *__restrict__ part, int with_diag) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < np; i += 256) {
    double v = A[i + (int64_t)np * j];
    if (i != j || with_diag) s = fma(v, v, s);
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[j] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) k_offnorm_final(const double *__restrict__ part, int np,
                                                       const double *__restrict__ fro,
                                                       double *__restrict__ off) {
  __shared__ double red[4];
  double s = 0;
  for (int j = threadIdx.x; j < np; j += 256) s += part[j];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0] + red[1] + red[2] + red[3];
    off[0] = fro ? (fro[0] > 0 ? sqrt(t) / fro[0] : 0.0) : sqrt(t);
  }
}

// Rotations of one round on the 32 x 32 principal submatrix of block pair k
// (local indices 0..15: block P, 16..31: block Q).  Every index pair (i, j)
// of the matrix is rotated exactly once per sweep, so a sweep is one cyclic
// Jacobi sweep in a block-parallel order: the round visits the 256 cross
// pairs (i in P, j in Q) in 16 sub-rounds of 16 disjoint rotations (i with
// 16 + (i + u) mod 16), and the first round of a sweep also visits the pairs
// within each block beforehand (15 sub-rounds, round-robin within P and Q).
// The tile is double-buffered in LDS: in a sub-round every thread reads the
// current tile, computes the two rotations of its 2 x 2 pair block itself
// and writes its four entries of the next tile; rows of J = prod R are
// updated in place; one barrier per sub-round.
__device__ __forceinline__ void sub_round_pair(int u, bool first, int k, int &p, int &q) {
  if (first && u < kJB - 1) {
    const int base = k < kJB / 2 ? 0 : kJB, kk = k & (kJB / 2 - 1);
    p = base + rr_player(kk, u, kJB);
    q = base + rr_player(kJB - 1 - kk, u, kJB);
  } else {
    const int sr = first ? u - (kJB - 1) : u;
    p = k;
    q = kJB + ((k + sr) & (kJB - 1));
  }
}

__global__ void __launch_bounds__(256) k_jacobi_solve(const double *__restrict__ A, int np, int nb,
                                                      int round, const double *__restrict__ fro,
                                                      double *__restrict__ Jout, int *cnt) {
  __shared__ double S[2][kJT][kJT + 1];
  __shared__ double Jm[kJT][kJT + 1];
  __shared__ int rot_any;
  const int k = blockIdx.x, tid = threadIdx.x;
  for (int e = tid; e < kJT * kJT; e += 256) {
    int i = e & 31, j = e >> 5;
    int gi = pair_index(k, i, round, nb), gj = pair_index(k, j, round, nb);
    S[0][i][j] = A[gi + (int64_t)np * gj];
    Jm[i][j] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) rot_any = 0;
  const double tol_abs = 1e-15 * fro[0], tol_rel = 1e-15;
  const int P1 = tid >> 4, P2 = tid & 15;
  const int jr = tid >> 4;   // J rows jr and jr + 16, column pair P2
  const bool first = round == 0;
  const int nsub = first ? 2 * kJB - 1 : kJB;
  int cur = 0;
  __syncthreads();
  for (int u = 0; u < nsub; ++u) {
    int p1, q1, p2, q2;
    sub_round_pair(u, first, P1, p1, q1);
    sub_round_pair(u, first, P2, p2, q2);
    const double a11 = S[cur][p1][p1], a12 = S[cur][q1][q1], a13 = S[cur][p1][q1];
    const double a21 = S[cur][p2][p2], a22 = S[cur][q2][q2], a23 = S[cur][p2][q2];
    const double b11 = S[cur][p1][p2], b12 = S[cur][p1][q2];
    const double b21 = S[cur][q1][p2], b22 = S[cur][q1][q2];
    double c1, s1, c2, s2;
    const bool r1 = jacobi_rotation(a11, a12, a13, tol_rel, tol_abs, c1, s1);
    const bool r2 = jacobi_rotation(a21, a22, a23, tol_rel, tol_abs, c2, s2);
    if (r2 && P1 == 0) rot_any = 1;
    const double t11 = c2 * b11 - s2 * b12, t12 = s2 * b11 + c2 * b12;
    const double t21 = c2 * b21 - s2 * b22, t22 = s2 * b21 + c2 * b22;
    double n11 = c1 * t11 - s1 * t21, n12 = c1 * t12 - s1 * t22;
    double n21 = s1 * t11 + c1 * t21, n22 = s1 * t12 + c1 * t22;
    if (P1 == P2 && r1) {
      n12 = 0.0;
      n21 = 0.0;
    }
    const int nx = cur ^ 1;
    S[nx][p1][p2] = n11;
    S[nx][p1][q2] = n12;
    S[nx][q1][p2] = n21;
    S[nx][q1][q2] = n22;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = jr + 16 * h;
      const double jp = Jm[row][p2], jq = Jm[row][q2];
      Jm[row][p2] = c2 * jp - s2 * jq;
      Jm[row][q2] = s2 * jp + c2 * jq;
    }
    cur = nx;
    __syncthreads();
  }
  double *Jo = Jout + (int64_t)k * kJT * kJT;
  for (int e = tid; e < kJT * kJT; e += 256) {
    int i = e & 31, j = e >> 5;
    Jo[i + kJT * j] = Jm[i][j];
  }
  if (tid == 0 && rot_any) atomicAdd(cnt, 1);
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Apply the round's rotations: every 32 x 32 tile of A (rows of block pair
// k1, columns of pair k2) becomes J_k1^T A J_k2, and every 32-row tile of V
// becomes V J_k2.  Both products run on the FP64 matrix cores, one 16 x 16
// output quarter per wavefront (v_mfma_f64_16x16x4f64: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; result register r is
// D[l / 16 + 4 r][l % 16]).
__global__ void __launch_bounds__(256) k_jacobi_update(double *__restrict__ A, double *__restrict__ V,
                                                       int np, int nb, int round,
                                                       const double *__restrict__ Jbuf) {
  __shared__ double Tl[kJT][kJT + 1];
  __shared__ double J1[kJT][kJT + 1];
  __shared__ double J2[kJT][kJT + 1];
  __shared__ double Tm[kJT][kJT + 1];
  const int npair = nb / 2;
  const int tilesA = npair * npair;
  int w = blockIdx.x;
  const int tid = threadIdx.x;
  bool isA = w < tilesA;
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
  for (int e = tid; e < kJT * kJT; e += 256) {
    int i = e & 31, j = e >> 5;
    int gj = pair_index(k2, j, round, nb);
    if (isA) {
      int gi = pair_index(k1, i, round, nb);
      Tl[i][j] = A[gi + (int64_t)np * gj];
      J1[i][j] = Jbuf[(int64_t)k1 * kJT * kJT + i + kJT * j];
    } else {
      Tl[i][j] = V[rc0 + i + (int64_t)np * gj];
    }
    J2[i][j] = Jbuf[(int64_t)k2 * kJT * kJT + i + kJT * j];
  }
  __syncthreads();
  const int wv = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
  const int ti = wv >> 1, tj = wv & 1;   // this wave's 16 x 16 output quarter
  v4d acc = {0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < 8; ++kk)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Tl[16 * ti + lr][4 * kk + lk],
                                               J2[4 * kk + lk][16 * tj + lr], acc, 0, 0, 0);
  if (!isA) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * ti + lk + 4 * r, j = 16 * tj + lr;
      V[rc0 + i + (int64_t)np * pair_index(k2, j, round, nb)] = acc[r];
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) Tm[16 * ti + lk + 4 * r][16 * tj + lr] = acc[r];
  __syncthreads();
  acc = v4d{0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < 8; ++kk)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(J1[4 * kk + lk][16 * ti + lr],
                                               Tm[4 * kk + lk][16 * tj + lr], acc, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 16 * ti + lk + 4 * r, j = 16 * tj + lr;
    A[pair_index(k1, i, round, nb) + (int64_t)np * pair_index(k2, j, round, nb)] = acc[r];
  }
}

// Eigenvalues from the diagonal, ranked in descending order (ties by index).
__global__ void __launch_bounds__(1024) k_eig_rank(const double *__restrict__ Ap, int np, int n,
                                                   double *__restrict__ w, int *__restrict__ rank) {
  for (int i = threadIdx.x; i < n; i += 1024) {
    double li = Ap[i + (int64_t)np * i];
    int r = 0;
    for (int j = 0; j < n; ++j) {
      double lj = Ap[j + (int64_t)np * j];
      r += (lj > li) || (lj == li && j < i);
    }
    w[r] = li;
    rank[i] = r;
  }
}

__global__ void k_eig_vecs(const double *__restrict__ V, int np, int n, const int *__restrict__ rank,
                           double *__restrict__ W, int64_t ldw) {
  int r = blockIdx.y * blockDim.x + threadIdx.x;
  int i = blockIdx.x;
  if (r < n) W[r + ldw * rank[i]] = V[r + (int64_t)np * i];
}

EigWork::~EigWork() {
  if (cnt_host) (void)hipHostFree(cnt_host);
}

int sym_eig(const double *A, int64_t lda, int n, double *w, double *W, int64_t ldw,
            hipStream_t st, EigWork &ws) {
  if (n <= 0) return 0;
  const int np = (n + kJT - 1) / kJT * kJT;
  const int nb = np / kJB;
  const int npair = nb / 2;
  ws.A.reserve((size_t)np * np);
  ws.V.reserve((size_t)np * np);
  ws.J.reserve((size_t)npair * kJT * kJT);
  ws.fro.reserve(2 + np);   // ||A||_F, relative off-diagonal norm, column partials
  ws.cnt.reserve(1 + np);   // counter + rank scratch
  if (!ws.cnt_host) FKF_CHECK_HIP(hipHostMalloc((void **)&ws.cnt_host, sizeof(double)));
  int64_t tot = (int64_t)np * np;
  hipLaunchKernelGGL(k_jacobi_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, A, lda,
                     n, np, ws.A.p, ws.V.p);
  hipLaunchKernelGGL(k_offnorm_cols, dim3(np), dim3(256), 0, st, ws.A.p, np, ws.fro.p + 2, 1);
  hipLaunchKernelGGL(k_offnorm_final, dim3(1), dim3(256), 0, st, ws.fro.p + 2, np,
                     (const double *)nullptr, ws.fro.p);
  const unsigned grid_upd = (unsigned)(npair * npair + (np / kJT) * npair);
  // Stop when the relative off-diagonal norm is below 1e-12 (a perturbation of
  // at most 1e-12 ||A||_F on the eigenvalues) or a sweep rotates nothing.
  int sweeps = 0;
  double *off_host = reinterpret_cast<double *>(ws.cnt_host);
  for (int sw = 0; sw < 40; ++sw) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, ws.cnt.p, 0);
    for (int r = 0; r < nb - 1; ++r) {
      {
        FKF_TRACE("eig_jacobi_solve", st);
        hipLaunchKernelGGL(k_jacobi_solve, dim3(npair), dim3(256), 0, st, ws.A.p, np, nb, r,
                           ws.fro.p, ws.J.p, ws.cnt.p);
      }
      {
        FKF_TRACE("eig_jacobi_update", st);
        hipLaunchKernelGGL(k_jacobi_update, dim3(grid_upd), dim3(256), 0, st, ws.A.p, ws.V.p, np,
                           nb, r, ws.J.p);
      }
    }
    hipLaunchKernelGGL(k_offnorm_cols, dim3(np), dim3(256), 0, st, ws.A.p, np, ws.fro.p + 2, 0);
    hipLaunchKernelGGL(k_offnorm_final, dim3(1), dim3(256), 0, st, ws.fro.p + 2, np, ws.fro.p,
                       ws.fro.p + 1);
    FKF_CHECK_HIP(hipMemcpyAsync(off_host, ws.fro.p + 1, sizeof(double), hipMemcpyDeviceToHost, st));
    int rotated = 0;
    FKF_CHECK_HIP(hipMemcpyAsync(&rotated, ws.cnt.p, sizeof(int), hipMemcpyDeviceToHost, st));
    FKF_CHECK_HIP(hipStreamSynchronize(st));
    ++sweeps;
    if (*off_host <= 1e-12 || rotated == 0) break;
  }
  int *rank = ws.cnt.p + 1;
  hipLaunchKernelGGL(k_eig_rank, dim3(1), dim3(1024), 0, st, ws.A.p, np, n, w, rank);
  hipLaunchKernelGGL(k_eig_vecs, dim3(n, (unsigned)((n + 255) / 256)), dim3(256), 0, st, ws.V.p,
                     np, n, rank, W, ldw);
  FKF_CHECK_HIP(hipGetLastError());
  return sweeps;
}

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

// G[m, j] = H_m . P[:, j]: one wavefront per entry, lanes split the row's nnz.
__global__ void __launch_bounds__(256) k_gram_hp(const int64_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col,
                                                 const double *__restrict__ val, int n_m, int64_t n,
                                                 const double *__restrict__ P,
                                                 double *__restrict__ G) {
  int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= (int64_t)n_m * n_m) return;
  int m = (int)(e % n_m), j = (int)(e / n_m);
  int l = threadIdx.x & 63;
  const double *Pj = P + n * j;
  double s = 0;
  for (int64_t q = rowptr[m] + l; q < rowptr[m + 1]; q += 64) s = fma(val[q], Pj[col[q]], s);
  s = wave_sum(s);
  if (l == 0) G[m + (int64_t)n_m * j] = s;
}

__global__ void k_gram_sym(const double *__restrict__ G, int n_m, const double *__restrict__ r,
                           double *__restrict__ A) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n_m * n_m) return;
  int m = (int)(e % n_m), j = (int)(e / n_m);
  A[e] = 0.5 * (G[e] + G[j + (int64_t)n_m * m]) / sqrt(r[m] * r[j]);
}

void innovation_gram(const int64_t *rowptr, const int32_t *col, const double *val, int n_m,
                     int64_t n, const double *P, const double *noise_var, double *G, double *A,
                     hipStream_t st) {
  int64_t e = (int64_t)n_m * n_m;
  if (e == 0) return;
  hipLaunchKernelGGL(k_gram_hp, dim3((unsigned)((e + 3) / 4)), dim3(256), 0, st, rowptr, col, val,
                     n_m, n, P, G);
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

void gemm_nn(int64_t m, int n, int k, const double *A, int64_t lda, const double *B, int64_t ldb,
             double *C, int64_t ldc, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
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
  const int64_t tm = (m + 63) / 64, tn = (n + 63) / 64;
  int splits = 1;
  if (work && tm * tn < 256 && k >= 1024) {
    splits = (int)std::min<int64_t>((256 + tm * tn - 1) / (tm * tn), k / 512);
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
// S (m x m, ld m) = L L^T in place (lower), then x = S^-1 b overwriting b.
// One workgroup; right-looking, column by column.  A non-positive pivot sets
// *err = FKF_E_NOT_SPD and leaves b unchanged.
__global__ void __launch_bounds__(1024) k_chol_solve(double *__restrict__ S, int m,
                                                     double *__restrict__ b, int *err) {
  __shared__ double piv;
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    if (tid == 0) {
      double d = S[j + (int64_t)m * j];
      if (!(d > 0.0) || !isfinite(d)) {
        bad = 1;
        piv = 1.0;
      } else {
        piv = sqrt(d);
      }
      S[j + (int64_t)m * j] = piv;
    }
    __syncthreads();
    if (bad) break;
    const double ip = 1.0 / piv;
    for (int i = j + 1 + tid; i < m; i += 1024) S[i + (int64_t)m * j] *= ip;
    __syncthreads();
    // trailing update of the lower triangle
    const int r = m - j - 1;
    const int64_t tot = (int64_t)r * (r + 1) / 2;
    for (int64_t e = tid; e < tot; e += 1024) {
      // e -> (i, k) with 0 <= k <= i < r, column-wise packing
      int64_t kk = (int64_t)((sqrt(8.0 * (double)e + 1.0) - 1.0) / 2.0);
      while (kk * (kk + 1) / 2 > e) --kk;
      while ((kk + 1) * (kk + 2) / 2 <= e) ++kk;
      int64_t i = kk, c = e - kk * (kk + 1) / 2;   // row index i >= column index c
      int gi = j + 1 + (int)i, gc = j + 1 + (int)c;
      S[gi + (int64_t)m * gc] -= S[gi + (int64_t)m * j] * S[gc + (int64_t)m * j];
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) atomicExch(err, (int)FKF_E_NOT_SPD);
    return;
  }
  // forward: L y = b
  for (int j = 0; j < m; ++j) {
    if (tid == 0) b[j] /= S[j + (int64_t)m * j];
    __syncthreads();
    const double yj = b[j];
    for (int i = j + 1 + tid; i < m; i += 1024) b[i] -= S[i + (int64_t)m * j] * yj;
    __syncthreads();
  }
  // backward: L^T x = y
  for (int j = m - 1; j >= 0; --j) {
    if (tid == 0) b[j] /= S[j + (int64_t)m * j];
    __syncthreads();
    const double xj = b[j];
    for (int i = tid; i < j; i += 1024) b[i] -= S[j + (int64_t)m * i] * xj;
    __syncthreads();
  }
}

void chol_solve(double *S, int m, double *b, int *err, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(1024), 0, st, S, m, b, err);
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
