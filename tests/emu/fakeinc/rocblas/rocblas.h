// CPU stand-in for the rocBLAS calls of the reinversion (column-major, naive loops).
#pragma once
#include "../../emu_hip.h"
typedef struct emu_blas* rocblas_handle;
typedef enum { rocblas_status_success = 0, rocblas_status_memory_error = 5 } rocblas_status;
typedef enum { rocblas_operation_none = 111, rocblas_operation_transpose = 112 } rocblas_operation;
typedef enum { rocblas_fill_upper = 121, rocblas_fill_lower = 122 } rocblas_fill;
typedef enum { rocblas_diagonal_non_unit = 131, rocblas_diagonal_unit = 132 } rocblas_diagonal;
typedef enum { rocblas_side_left = 141, rocblas_side_right = 142 } rocblas_side;
typedef enum { rocblas_atomics_not_allowed = 0, rocblas_atomics_allowed = 1 } rocblas_atomics_mode;
inline void rocblas_initialize() {}
inline rocblas_status rocblas_create_handle(rocblas_handle* h) { *h = (rocblas_handle)0x1; return rocblas_status_success; }
inline rocblas_status rocblas_destroy_handle(rocblas_handle) { return rocblas_status_success; }
inline rocblas_status rocblas_set_stream(rocblas_handle, hipStream_t) { return rocblas_status_success; }
inline rocblas_status rocblas_set_atomics_mode(rocblas_handle, rocblas_atomics_mode) { return rocblas_status_success; }
inline const char* rocblas_status_to_string(rocblas_status) { return "emu"; }
inline rocblas_status rocblas_dgemm(rocblas_handle, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
                                    const double* alpha, const double* A, int lda, const double* B, int ldb,
                                    const double* beta, double* C, int ldc) {
  if (ta != rocblas_operation_none || tb != rocblas_operation_none) abort();
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      for (int p = 0; p < k; ++p) s += A[i + (size_t)p * lda] * B[p + (size_t)j * ldb];
      double& c = C[i + (size_t)j * ldc];
      c = (*beta == 0.0 ? 0.0 : *beta * c) + *alpha * s;
    }
  return rocblas_status_success;
}
inline rocblas_status rocblas_dtrsm(rocblas_handle, rocblas_side side, rocblas_fill fill, rocblas_operation op,
                                    rocblas_diagonal diag, int m, int n, const double* alpha, const double* A, int lda,
                                    double* B, int ldb) {
  if (side != rocblas_side_left || op != rocblas_operation_none) abort();
  for (int j = 0; j < n; ++j) {
    double* x = B + (size_t)j * ldb;
    for (int i = 0; i < m; ++i) x[i] *= *alpha;
    if (fill == rocblas_fill_lower)
      for (int i = 0; i < m; ++i) {
        double s = x[i];
        for (int p = 0; p < i; ++p) s -= A[i + (size_t)p * lda] * x[p];
        x[i] = diag == rocblas_diagonal_unit ? s : s / A[i + (size_t)i * lda];
      }
    else
      for (int i = m - 1; i >= 0; --i) {
        double s = x[i];
        for (int p = i + 1; p < m; ++p) s -= A[i + (size_t)p * lda] * x[p];
        x[i] = diag == rocblas_diagonal_unit ? s : s / A[i + (size_t)i * lda];
      }
  }
  return rocblas_status_success;
}
