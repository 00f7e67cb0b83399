// FP64 level-3 kernels of the reinversion (gfx950): a matrix product on the FP64 matrix
// cores and a blocked triangular solve built on it.  Column-major throughout.
//
// k_dgemm computes C = beta C - A B (beta 0 or 1) for an M x K matrix A and a K x N matrix
// B.  A workgroup of four wavefronts owns a 64 x 64 tile of C; each wavefront a 32 x 32
// quarter, held as 2 x 2 accumulators of v_mfma_f64_16x16x4f64 (16 x 16 outputs, 4 doubles
// per lane).  A and B move through LDS in slices of 16 along K, double-buffered: the next
// slice's global loads are issued before the current slice's MFMAs, and stored into the
// other LDS buffer after them.  Out-of-range rows, columns and K are read as zeros and
// never written.  Every output sums its K products in one fixed order, so the result does
// not depend on timing.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lp_gemm.h"

namespace lpgpu {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kTM = 64, kTN = 64, kTK = 16, kThreads = 256;
constexpr int kPadA = 4;  // row padding of the LDS tiles (doubles)

template <bool ACC>
__global__ __launch_bounds__(kThreads) void k_dgemm(int M, int N, int K, const double* __restrict__ A, int lda,
                                                    const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                    int ldc) {
  __shared__ double sA[2][kTK][kTM + kPadA];  // sA[buf][k][i]
  __shared__ double sB[2][kTK][kTN + kPadA];  // sB[buf][k][j]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.x * kTM, j0 = blockIdx.y * kTN;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  // loads: A rows i0 + (tid % 64), k = tid / 64 + 4u; B k = tid % 16, columns j0 + tid / 16 + 16u
  const int ai = i0 + (tid & 63), ak = tid >> 6;
  const int bk = tid & 15, bj = j0 + (tid >> 4);
  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k0 + ak + 4 * u;
      ra[u] = (ai < M && kk < K) ? A[(size_t)ai + (size_t)kk * lda] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k0 + bk, j = bj + 16 * u;
      rb[u] = (kk < K && j < N) ? B[(size_t)kk + (size_t)j * ldb] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) sA[buf][ak + 4 * u][tid & 63] = ra[u];
#pragma unroll
    for (int u = 0; u < 4; ++u) sB[buf][bk][(tid >> 4) + 16 * u] = rb[u];
  };
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  const int nk = (K + kTK - 1) / kTK;
  if (nk > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  const int r16 = lane & 15, kq = lane >> 4;
  for (int t = 0; t < nk; ++t) {
    const int buf = t & 1;
    if (t + 1 < nk) load((t + 1) * kTK);
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 4) {
      const double a0 = sA[buf][kk + kq][wr + r16];
      const double a1 = sA[buf][kk + kq][wr + 16 + r16];
      const double b0 = sB[buf][kk + kq][wc + r16];
      const double b1 = sB[buf][kk + kq][wc + 16 + r16];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (t + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }
  // accumulator layout: lane l, element r holds row 4 (l / 16) + r, column l % 16 of its tile
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wr + 16 * a + 4 * kq + r, col = j0 + wc + 16 * b + r16;
        if (row < M && col < N) {
          double* c = C + (size_t)row + (size_t)col * ldc;
          const double v = acc[a][b][r];
          *c = ACC ? *c - v : -v;
        }
      }
}

// X[J0:J0+nb, 0:ncol] := T^-1 X[J0:J0+nb, 0:ncol] for the diagonal block T = M[J0:J0+nb,
// J0:J0+nb] (nb <= kTrsmNb; leading dimensions ldm, ldx): unit lower triangular (forward
// substitution) or non-unit upper triangular (backward).  T is staged in LDS by every
// workgroup; each wavefront solves whole columns, lane l holding rows l and l + 64, the
// solved entry broadcast by readlane.
__device__ __forceinline__ double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <bool UPPER>
__global__ __launch_bounds__(256) void k_trsm_block(const double* __restrict__ Mt, int ldm, double* __restrict__ X,
                                                    int ldx, int J0, int nb, int ncol) {
  __shared__ double sT[kTrsmNb * kTrsmNb];  // column-major nb x nb
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int waves = 256 / 64;
  for (int e = tid; e < nb * nb; e += 256) sT[e] = Mt[(size_t)(J0 + e % nb) + (size_t)(J0 + e / nb) * ldm];
  __syncthreads();
  const int i0 = lane, i1 = lane + 64;
  for (int col = blockIdx.x * waves + wave; col < ncol; col += gridDim.x * waves) {
    double* xc = X + (size_t)J0 + (size_t)col * ldx;
    double b0 = i0 < nb ? xc[i0] : 0.0;
    double b1 = i1 < nb ? xc[i1] : 0.0;
    if (!UPPER) {
      for (int j = 0; j < nb; ++j) {
        const double xj = j < 64 ? read_lane(b0, j) : read_lane(b1, j - 64);
        const double l0 = i0 > j && i0 < nb ? sT[i0 + j * nb] : 0.0;
        const double l1 = i1 > j && i1 < nb ? sT[i1 + j * nb] : 0.0;
        b0 = fma(-l0, xj, b0);
        b1 = fma(-l1, xj, b1);
      }
    } else {
      for (int j = nb - 1; j >= 0; --j) {
        // x_j = b_j / U_jj, then b_i -= U_ij x_j for the rows above j
        const double d = sT[j + j * nb];
        if (i0 == j) b0 = b0 / d;
        if (i1 == j) b1 = b1 / d;
        const double xj = j < 64 ? read_lane(b0, j) : read_lane(b1, j - 64);
        const double u0 = i0 < j ? sT[i0 + j * nb] : 0.0;
        const double u1 = i1 < j ? sT[i1 + j * nb] : 0.0;
        b0 = fma(-u0, xj, b0);
        b1 = fma(-u1, xj, b1);
      }
    }
    if (i0 < nb) xc[i0] = b0;
    if (i1 < nb) xc[i1] = b1;
  }
}

}  // namespace

hipError_t launch_dgemm(int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                        bool accumulate, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const dim3 grid((M + kTM - 1) / kTM, (N + kTN - 1) / kTN);
  if (accumulate)
    hipLaunchKernelGGL(k_dgemm<true>, grid, dim3(kThreads), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  else
    hipLaunchKernelGGL(k_dgemm<false>, grid, dim3(kThreads), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  return hipGetLastError();
}

hipError_t launch_trsm(const double* T, int ldt, int k, double* X, int ldx, int ncol, bool upper, hipStream_t s) {
  if (k <= 0 || ncol <= 0) return hipSuccess;
  const int grid = std::max(1, std::min(1024, (ncol + 3) / 4));
  const int nblk = (k + kTrsmNb - 1) / kTrsmNb;
  for (int bi = 0; bi < nblk; ++bi) {
    // lower: blocks top to bottom; upper: bottom to top
    const int blk = upper ? nblk - 1 - bi : bi;
    const int J0 = blk * kTrsmNb, nb = std::min(kTrsmNb, k - J0);
    if (upper)
      hipLaunchKernelGGL(k_trsm_block<true>, dim3(grid), dim3(256), 0, s, T, ldt, X, ldx, J0, nb, ncol);
    else
      hipLaunchKernelGGL(k_trsm_block<false>, dim3(grid), dim3(256), 0, s, T, ldt, X, ldx, J0, nb, ncol);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the solved block row updates the rows still to be solved
    if (!upper && J0 + nb < k)
      e = launch_dgemm(k - J0 - nb, ncol, nb, T + (size_t)(J0 + nb) + (size_t)J0 * ldt, ldt, X + J0, ldx,
                       X + J0 + nb, ldx, true, s);
    else if (upper && J0 > 0)
      e = launch_dgemm(J0, ncol, nb, T + (size_t)J0 * ldt, ldt, X + J0, ldx, X, ldx, true, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lpgpu
