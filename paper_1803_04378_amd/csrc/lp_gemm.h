// FP64 level-3 kernels of the reinversion (lp_gemm.hip), column-major.
#pragma once
#include <hip/hip_runtime.h>

namespace lpgpu {

// Rows of one diagonal block of the blocked triangular solve (two per lane of a wavefront).
constexpr int kTrsmNb = 128;

// C = (accumulate ? C : 0) - A B, with A M x K (leading dimension lda), B K x N (ldb), C
// M x N (ldc); C must not overlap A or B.
hipError_t launch_dgemm(int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                        bool accumulate, hipStream_t s);

// X := T^-1 X for the k x k triangle of T (leading dimension ldt) and X k x ncol (ldx):
// unit lower triangular (upper = false) or non-unit upper triangular (upper = true);
// blocks of kTrsmNb rows solved in LDS, the rest of X updated by launch_dgemm.
hipError_t launch_trsm(const double* T, int ldt, int k, double* X, int ldx, int ncol, bool upper, hipStream_t s);

}  // namespace lpgpu
