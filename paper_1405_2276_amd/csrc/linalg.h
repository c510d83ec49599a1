// Host entry points of the dense/sparse linear-algebra kernels (linalg.hip).
#pragma once

#include "common.h"

namespace fkf {

// Workspace of the symmetric eigensolver (grown on demand).
struct EigWork {
  DevBuf<double> A, V, J, fro;
  DevBuf<int> cnt;
  int *cnt_host = nullptr;   // pinned host scratch (8 bytes)
  ~EigWork();
};

// Eigen-decomposition of a symmetric n x n FP64 matrix A (column-major, lda)
// by two-sided block Jacobi: w (n, descending) and W (n x n, column j the
// eigenvector of w[j], ldw).  Returns the number of sweeps used.  Synchronises
// the stream once per sweep to test convergence.
int sym_eig(const double *A, int64_t lda, int n, double *w, double *W, int64_t ldw,
            hipStream_t st, EigWork &ws);

// y (n_m) = H x for CSR H.
void spmv(const int64_t *rowptr, const int32_t *col, const double *val, int n_m,
          const double *x, double *y, hipStream_t st);

// D (n x n_m, column-major, ld n) = dense H^T.
void dense_ht(const int64_t *rowptr, const int32_t *col, const double *val, int n_m, int64_t n,
              double *D, hipStream_t st);

// A (n_m x n_m) = R^-1/2 sym(H P) R^-1/2 where P is n x n_m (ld n), R diagonal.
void innovation_gram(const int64_t *rowptr, const int32_t *col, const double *val, int n_m,
                     int64_t n, const double *P, const double *noise_var, double *G,
                     double *A, hipStream_t st);

// C (m x n) = A (m x k) * B (k x n), all column-major FP64.
void gemm_nn(int64_t m, int n, int k, const double *A, int64_t lda, const double *B, int64_t ldb,
             double *C, int64_t ldc, hipStream_t st);

// Scale row i of a column-major m x n matrix by s[i] (in place).
void scale_rows(int64_t m, int n, const double *s, double *A, int64_t lda, hipStream_t st);

void fill(double *p, int64_t n, double v, hipStream_t st);

}  // namespace fkf
