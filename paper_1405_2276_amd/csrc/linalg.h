// Host entry points of the dense/sparse linear-algebra kernels (linalg.hip).
#pragma once

#include "common.h"

namespace fkf {

// One symmetric eigenproblem of a batch: A (n x n, column-major, lda) in,
// eigenvalues w (n, descending) and eigenvectors W (n x n, ldw) out.
struct EigProblem {
  const double *A;
  int64_t lda;
  int32_t n, pad;
  double *w;
  double *W;
  int64_t ldw;
};

// Workspace of the symmetric eigensolver (grown on demand).
struct EigWork {
  DevBuf<double> A, A2, V, J, J2, fro;   // A, J double-buffered across rounds
  DevBuf<int> cnt;
  DevBuf<int32_t> pidx;       // pair index table of the rounds
  DevBuf<EigProblem> probs;   // descriptors of the batch
  int pidx_np = -1;
  int *cnt_host = nullptr;   // pinned host scratch (4 ints; [2]: convergence flag)
  hipEvent_t ev = nullptr;   // marks the convergence test of the last sweep
  // reduction + divide-and-conquer solver: merge tree of order dc_n (node,
  // wave and tile tables, launch ranges per tree height) and its arrays
  struct DcLevel {
    int node0, nodes, wave0, waves, tile0, tiles;
  };
  std::vector<DcLevel> dc_levels;
  int dc_n = -1;
  DevBuf<int32_t> dc_nodes, dc_wmap, dc_tiles;
  DevBuf<double> hv, Qc, Qp, U, dels, vec;
  DevBuf<int> ivec;
  ~EigWork();
};

// Eigen-decomposition of a symmetric n x n FP64 matrix A (column-major, lda):
// w (n, descending) and W (n x n, column j the eigenvector of w[j], ldw).
// Orders 3..1024 take sym_eig_dc (tol unused; returns 0); other orders take
// two-sided block Jacobi, stopped when the off-diagonal Frobenius norm is
// below tol ||A||_F, returning the number of sweeps (the stream is
// synchronised once per sweep to test convergence).
int sym_eig(const double *A, int64_t lda, int n, double *w, double *W, int64_t ldw,
            hipStream_t st, EigWork &ws, double tol = 1e-12, int *err = nullptr);

// Householder tridiagonalization + divide and conquer + back-transformation
// for 3 <= n <= 1024 (eig_dc.hip), same outputs as sym_eig.  A failure of the
// reduction's exchanges (its workgroups never all ran together) is latched
// into the device int *err as FKF_E_HIP (an existing error is kept); without
// err the stream is synchronised once and the failure thrown.
bool sym_eig_dc_supported(int n);
void sym_eig_dc(const double *A, int64_t lda, int n, double *w, double *W, int64_t ldw,
                hipStream_t st, EigWork &ws, int *err = nullptr);

// The same for count independent problems: one problem of a supported order
// takes sym_eig_dc (err as there; returns 0); otherwise block Jacobi in one
// sequence of launches (all padded to the largest order, one convergence flag
// each), returning the number of sweeps of the slowest problem.
int sym_eig_batched(const EigProblem *probs, int count, hipStream_t st, EigWork &ws,
                    double tol = 1e-12, int *err = nullptr);

// y (n_m) = H x for CSR H.
void spmv(const int64_t *rowptr, const int32_t *col, const double *val, int n_m,
          const double *x, double *y, hipStream_t st);

// D (n x n_m, column-major, ld n) = dense H^T.
void dense_ht(const int64_t *rowptr, const int32_t *col, const double *val, int n_m, int64_t n,
              double *D, hipStream_t st);

// G (n_m x n_m) = H P from its upper triangle (H Gamma H^T is symmetric) and
// A = R^-1/2 G R^-1/2, where P is n x n_m (ld n) and R diagonal.
void innovation_gram(const int64_t *rowptr, const int32_t *col, const double *val, int n_m,
                     int64_t n, const double *P, const double *noise_var, double *G,
                     double *A, hipStream_t st);

// C (m x n) = A (m x k) * B (k x n), all column-major FP64.
void gemm_nn(int64_t m, int n, int k, const double *A, int64_t lda, const double *B, int64_t ldb,
             double *C, int64_t ldc, hipStream_t st);

// Scale row i of a column-major m x n matrix by s[i] (in place).
void scale_rows(int64_t m, int n, const double *s, double *A, int64_t lda, hipStream_t st);

void fill(double *p, int64_t n, double v, hipStream_t st);

// C = alpha op(A) op(B) + beta C (FP64, column-major; op = transpose when the
// flag is set).  When work is given and the output has few tiles, the k range
// is split across workgroups and the slices are summed in a fixed order.
void gemm(bool ta, bool tb, int64_t m, int64_t n, int64_t k, double alpha, const double *A,
          int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
          hipStream_t st, DevBuf<double> *work);

// out (n_m x cols, ld n_m) = H X for CSR H and dense X (n x cols, ld ldx).
void sp_dense(const int64_t *rowptr, const int32_t *col, const double *val, int n_m,
              const double *X, int64_t ldx, int cols, double *out, hipStream_t st);

// In-place Cholesky of the SPD m x m matrix S (ld m, lower triangle used;
// the upper triangle is overwritten) and solve S x = b (b overwritten).
// flag: one device int of scratch.  Sets *err = FKF_E_NOT_SPD on a
// non-positive pivot and then leaves b unchanged.  With ll_acc (device),
// adds the Gaussian log-density -(b^T S^-1 b + log det S + m log 2 pi)/2 of
// the right-hand side to ll_acc[0].
void chol_solve(double *S, int m, double *b, int *flag, int *err, hipStream_t st,
                double *ll_acc = nullptr);

void scale_cols(int64_t m, int n, const double *s, double *A, int64_t lda, hipStream_t st);
void symmetrize(double *A, int m, hipStream_t st);
void scale2d(int64_t m, int n, double a, double *A, int64_t lda, hipStream_t st);
void copy2d(int64_t m, int n, const double *A, int64_t lda, double *B, int64_t ldb, hipStream_t st);

}  // namespace fkf
