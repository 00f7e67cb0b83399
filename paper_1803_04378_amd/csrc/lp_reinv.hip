// Reinversion of the basis in FP64 (gfx950).
//
// With the slacks of the rows in S basic, order the basis as (structural columns K,
// slack columns of S) and the rows as (R = rows whose slack is nonbasic, then S):
//     B = [ B11  0 ]      B^-1 = [  B11^-1        0 ]
//         [ B21  I ],            [ -B21 B11^-1    I ],
// with B11 = A'[R, K] (order k = |K| = |R|) and B21 = A'[S, K].  Only B11 is factorised:
//   1. gather G = [B11^T | B21^T] (k x m, column-major) from A';
//   2. LU with partial pivoting of M = B11^T, blocked right-looking: each panel is
//      factorised by one workgroup holding the panel in registers (the pivot search is a
//      chain of k dependent reductions, so it stays inside one workgroup), a second kernel
//      applies the panel's row interchanges to the other columns and forms
//      U12 = L11^-1 A12, and the trailing update A22 -= L21 U12 is a DGEMM;
//   3. X = M^-1 = U^-1 L^-1 P (two triangular solves on X = P), so that row b of B11^-1
//      is column b of X, contiguous;
//   4. C^T = -X B21^T (DGEMM): row s of -B21 B11^-1 is column s of C^T;
//   5. B^-1 written row by row in its row-major layout, x_B = B^-1 b, W = chat_B^T B^-1
//      and z = chat_B^T x_B from X and C^T.
// The DGEMMs and triangular solves are rocBLAS calls on the handle's stream (atomics off,
// so results are reproducible); everything else is below.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lp_reinv.h"
#include "lpgpu.h"

namespace lpgpu {

int record_error(int code, const std::string& msg);

struct ReinvState {
  rocblas_handle blas = nullptr;
  double* G = nullptr;
  size_t G_cap = 0;
  double* X = nullptr;
  size_t X_cap = 0;
  double* C = nullptr;
  size_t C_cap = 0;
  double* part = nullptr;
  size_t part_cap = 0;
  int32_t* idx = nullptr;  // kcol (k) | kpos (k) | rowlist (m) | rinfo (m) | colmap (ld)
  size_t idx_cap = 0;
  int32_t* aux = nullptr;  // rowperm (m) | interchange list (kPairs dst, kPairs src, count) | info
  size_t aux_cap = 0;
  int32_t* h_idx = nullptr;  // pinned
  size_t h_idx_cap = 0;
  int32_t* h_basis = nullptr;  // pinned
  size_t h_basis_cap = 0;
};

namespace {

constexpr int kPairs = 64;  // row interchanges of one panel touch at most 2 * 32 rows
constexpr int kRowPanelThreads = 256;
constexpr int kWChunk = 64;  // b-range of one partial sum of W

// G[b + a*k] = A'[rowlist[a], kcol[b]] for b < k, a < m, through a 32 x 32 LDS tile so that
// both the reads (down a column of A') and the writes (down a column of G) coalesce.
__global__ void k_gather(const double* __restrict__ A, int ld, const int32_t* __restrict__ kcol,
                         const int32_t* __restrict__ rowlist, int k, int m, double* __restrict__ G) {
  __shared__ double tile[32][33];
  const int a0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int yy = ty; yy < 32; yy += 8) {
    const int a = a0 + tx, b = b0 + yy;
    double v = 0.0;
    if (a < m && b < k) v = A[(size_t)rowlist[a] + (size_t)kcol[b] * ld];
    tile[yy][tx] = v;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int b = b0 + tx, a = a0 + yy;
    if (a < m && b < k) G[(size_t)b + (size_t)a * k] = tile[tx][yy];
  }
}

__global__ void k_reinv_setup(int32_t* rowperm, int k, int32_t* info) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) rowperm[i] = i;
  if (i == 0) *info = 0;
}

// Factorises the panel M[j0:k, j0:j0+jb] in place (jb <= JB): thread t of NT holds rows
// t, t + NT, ... (relative to j0) of the panel in registers.  Each column: the pivot is
// the row of largest |value| at or below the diagonal (lowest row on ties), rows c and p
// are exchanged through LDS, and the rows below are eliminated.  Rows keep a tag of the
// row they started the panel in; at the end the moved rows are listed as (dst, src)
// pairs for k_lu_rowpanel.  A zero (or NaN) pivot column sets *info.
template <int NT, int JB>
struct PanelShared {
  double u[JB], w[JB];
  double red_v[NT / 64];
  int red_i[NT / 64];
  int uo, wo, np;
};

// Column C of the panel; the column index is a template argument so that every access to
// the register-held rows is static.
template <int NT, int RPT, int JB, int C>
__device__ __forceinline__ void lu_column(double (&a)[RPT][JB], int (&org)[RPT], PanelShared<NT, JB>& sh, int R,
                                          int jb, bool& singular) {
  if constexpr (C < JB) {
    if (C < jb) {
      constexpr int W = NT / 64;
      const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
      double bv = -1.0;
      int bi = INT_MAX;
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int rho = tid + s * NT;
        if (rho >= C && rho < R) {
          const double v = fabs(a[s][C]);
          if (v > bv) {
            bv = v;
            bi = rho;
          }
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        sh.red_v[wave] = bv;
        sh.red_i[wave] = bi;
      }
      __syncthreads();
      bv = sh.red_v[0];
      bi = sh.red_i[0];
#pragma unroll
      for (int w = 1; w < W; ++w) {
        const double ov = sh.red_v[w];
        const int oi = sh.red_i[w];
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      const bool ok = bv > 0.0;
      if (!ok) singular = true;
      const int p = ok ? bi : C;
      // Row p to LDS.  Selects over every slot (rather than a branch on the owning slot)
      // keep all register indices static.
      {
        double uv[JB];
        int uo = 0;
        bool mine = false;
#pragma unroll
        for (int cc = 0; cc < JB; ++cc) uv[cc] = 0.0;
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const bool hit = tid + s * NT == p;
#pragma unroll
          for (int cc = 0; cc < JB; ++cc) uv[cc] = hit ? a[s][cc] : uv[cc];
          uo = hit ? org[s] : uo;
          mine = mine || hit;
        }
        if (mine) {
#pragma unroll
          for (int cc = 0; cc < JB; ++cc) sh.u[cc] = uv[cc];
          sh.uo = uo;
        }
      }
      if (tid == C) {  // row C < JB is slot 0 of thread C
#pragma unroll
        for (int cc = 0; cc < JB; ++cc) sh.w[cc] = a[0][cc];
        sh.wo = org[0];
      }
      __syncthreads();
      if (p != C) {
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const bool hit = tid + s * NT == p;
#pragma unroll
          for (int cc = 0; cc < JB; ++cc) a[s][cc] = hit ? sh.w[cc] : a[s][cc];
          org[s] = hit ? sh.wo : org[s];
        }
        if (tid == C) {
#pragma unroll
          for (int cc = 0; cc < JB; ++cc) a[0][cc] = sh.u[cc];
          org[0] = sh.uo;
        }
      }
      // Multipliers by one reciprocal of the pivot (as LAPACK's unblocked LU does).
      const double rpiv = 1.0 / sh.u[C];
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int rho = tid + s * NT;
        if (rho > C && rho < R) {
          const double l = a[s][C] * rpiv;
          a[s][C] = l;
#pragma unroll
          for (int cc = C + 1; cc < JB; ++cc) a[s][cc] = fma(-l, sh.u[cc], a[s][cc]);
        }
      }
      __syncthreads();
    }
    lu_column<NT, RPT, JB, C + 1>(a, org, sh, R, jb, singular);
  }
}

template <int NT, int RPT, int JB>
__global__ __launch_bounds__(NT) void k_lu_panel(double* __restrict__ M, int ld, int k, int j0, int jb,
                                                 int32_t* __restrict__ pairs, int32_t* __restrict__ info) {
  __shared__ PanelShared<NT, JB> sh;
  const int R = k - j0, tid = threadIdx.x;
  double a[RPT][JB];
  int org[RPT];
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int rho = tid + s * NT;
    org[s] = rho;
#pragma unroll
    for (int c = 0; c < JB; ++c)
      a[s][c] = (rho < R && c < jb) ? M[(size_t)(j0 + rho) + (size_t)(j0 + c) * ld] : 0.0;
  }
  if (tid == 0) sh.np = 0;
  bool singular = false;
  lu_column<NT, RPT, JB, 0>(a, org, sh, R, jb, singular);
  // Opaque copies: the store addresses are formed here, not kept live from the loads.
  int tid2 = tid, ld2 = ld;
  asm volatile("" : "+v"(tid2));
  asm volatile("" : "+s"(ld2));
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int rho = tid2 + s * NT;
    if (rho < R) {
#pragma unroll
      for (int c = 0; c < JB; ++c)
        if (c < jb) M[(size_t)(j0 + rho) + (size_t)(j0 + c) * ld2] = a[s][c];
      if (org[s] != rho) {
        const int q = atomicAdd(&sh.np, 1);
        pairs[q] = j0 + rho;
        pairs[kPairs + q] = j0 + org[s];
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    pairs[2 * kPairs] = sh.np;
    if (singular) *info = 1;
  }
}

// The panel's row interchanges applied to every column outside the panel and to the row
// permutation (the extra last "column"), then U12 = L11^-1 A12 by forward substitution
// (unit lower L11 staged in LDS) for the columns right of the panel.  One wavefront per
// column: lane q moves interchange pair q, and lane r holds row j0 + r of the column
// during the substitution.
constexpr int kRowPanelWaves = kRowPanelThreads / 64;

__global__ __launch_bounds__(kRowPanelThreads) void k_lu_rowpanel(double* __restrict__ M, int ld, int k, int j0,
                                                                  int jb, const int32_t* __restrict__ pairs,
                                                                  int32_t* __restrict__ rowperm) {
  __shared__ double s_l[32 * 32];
  const int np = pairs[2 * kPairs];
  for (int e = threadIdx.x; e < 32 * 32; e += kRowPanelThreads) {
    const int r = e / 32, c = e % 32;
    s_l[e] = (c < r && r < jb) ? M[(size_t)(j0 + r) + (size_t)(j0 + c) * ld] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int dst = lane < np ? pairs[lane] : 0;
  const int src = lane < np ? pairs[kPairs + lane] : 0;
  const int ncols = k - jb + 1;
  const int gw = blockIdx.x * kRowPanelWaves + (threadIdx.x >> 6);
  const int nw = gridDim.x * kRowPanelWaves;
  for (int e = gw; e < ncols; e += nw) {
    if (e == ncols - 1) {
      const int v = lane < np ? rowperm[src] : 0;
      __builtin_amdgcn_wave_barrier();
      if (lane < np) rowperm[dst] = v;
      continue;
    }
    const int col = e < j0 ? e : e + jb;
    double* colp = M + (size_t)col * ld;
    const double v = lane < np ? colp[src] : 0.0;
    __builtin_amdgcn_wave_barrier();
    if (lane < np) colp[dst] = v;
    if (col >= j0 + jb) {
      // Reads after this wave's own writes above: same wavefront, program order.
      double u = lane < jb ? colp[j0 + lane] : 0.0;
      for (int c = 0; c + 1 < jb; ++c) {
        const double uc = __shfl(u, c);
        if (lane > c && lane < jb) u = fma(-s_l[lane * 32 + c], uc, u);
      }
      if (lane < jb) colp[j0 + lane] = u;
    }
  }
}

// X = P: X[c, rowperm[c]] = 1 (column-major k x k).
__global__ void k_perm_matrix(double* __restrict__ X, int k, const int32_t* __restrict__ rowperm) {
  const size_t total = (size_t)k * k;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += stride) {
    const int r = (int)(e % k), col = (int)(e / k);
    X[e] = rowperm[r] == col ? 1.0 : 0.0;
  }
}

// B^-1 in its m x ld row-major layout.  Row p is the basis position: rinfo[p] = b >= 0 for
// the structural column kcol[b] (row b of B11^-1 = column b of X), or -(s+1) for the slack
// of row srow[s] (row s of -B21 B11^-1 = column s of C^T, plus the unit entry).
__global__ void k_reinv_scatter(double* __restrict__ Binv, int m, int ld, int k, const int32_t* __restrict__ rinfo,
                                const int32_t* __restrict__ colmap, const int32_t* __restrict__ srow,
                                const double* __restrict__ X, const double* __restrict__ Ct,
                                const int32_t* __restrict__ info) {
  if (*info) return;
  const size_t total = (size_t)m * ld;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += stride) {
    const int p = (int)(e / ld), j = (int)(e % ld);
    const int a = colmap[j];
    const int ri = rinfo[p];
    double v;
    if (ri >= 0) {
      v = a >= 0 ? X[(size_t)a + (size_t)ri * k] : 0.0;
    } else {
      const int s = -ri - 1;
      v = a >= 0 ? Ct[(size_t)a + (size_t)s * k] : (j == srow[s] ? 1.0 : 0.0);
    }
    Binv[e] = v;
  }
}

// x_B = B^-1 b, one wavefront per basis position (lane fma chains + xor butterfly).
__global__ void k_reinv_xb(double* __restrict__ xB, int m, int k, const int32_t* __restrict__ rinfo,
                           const int32_t* __restrict__ rowlist, const double* __restrict__ X,
                           const double* __restrict__ Ct, const double* __restrict__ b, double eps_z,
                           const int32_t* __restrict__ info) {
  if (*info) return;
  const int lane = threadIdx.x & 63;
  const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nw = (gridDim.x * blockDim.x) >> 6;
  for (int p = gw; p < m; p += nw) {
    const int ri = rinfo[p];
    const double* col = ri >= 0 ? X + (size_t)ri * k : Ct + (size_t)(-ri - 1) * k;
    double acc = 0.0;
    for (int a = lane; a < k; a += 64) acc = fma(col[a], b[rowlist[a]], acc);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) {
      double x = ri >= 0 ? acc : b[rowlist[k + (-ri - 1)]] + acc;
      if (fabs(x) < eps_z) x = 0.0;
      xB[p] = x;
    }
  }
}

// W_j = sum_b chat_{kcol[b]} X[a, b] for j = rowlist[a] (a < k), 0 elsewhere: partial sums
// over b-chunks of kWChunk, then their sum in chunk order.
__global__ void k_reinv_w_part(double* __restrict__ part, int ld, int k, const int32_t* __restrict__ colmap,
                               const int32_t* __restrict__ kcol, const double* __restrict__ chat,
                               const double* __restrict__ X, const int32_t* __restrict__ info) {
  if (*info) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  if (j >= ld) return;
  const int a = colmap[j];
  double acc = 0.0;
  if (a >= 0) {
    const int b1 = min(k, (chunk + 1) * kWChunk);
    for (int b = chunk * kWChunk; b < b1; ++b) acc = fma(chat[kcol[b]], X[(size_t)a + (size_t)b * k], acc);
  }
  part[(size_t)chunk * ld + j] = acc;
}

__global__ void k_reinv_w_sum(double* __restrict__ W, const double* __restrict__ part, int ld, int nchunk,
                              const int32_t* __restrict__ info) {
  if (*info) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ld) return;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += part[(size_t)c * ld + j];
  W[j] = acc;
}

// z = chat_B^T x_B over the structural basic variables, then the control block: the new
// B^-1 already reflects the last pivot, so no row update is pending any more.
__global__ __launch_bounds__(1024) void k_reinv_finish(Ctrl* ctl, int k, const int32_t* __restrict__ kcol,
                                                       const int32_t* __restrict__ kpos,
                                                       const double* __restrict__ chat,
                                                       const double* __restrict__ xB,
                                                       const int32_t* __restrict__ info) {
  __shared__ double red[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double acc = 0.0;
  for (int b = tid; b < k; b += 1024) acc = fma(chat[kcol[b]], xB[kpos[b]], acc);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (tid == 0) {
    double z = 0.0;
    for (int w = 0; w < 16; ++w) z += red[w];
    if (*info == 0) {
      ctl->z = z;
      ctl->r = -1;
      ctl->n_reinv += 1;
    } else {
      ctl->n_reinv_failed += 1;
    }
  }
}

template <class T>
hipError_t grow(T** ptr, size_t* cap, size_t need) {
  if (need <= *cap && *ptr) return hipSuccess;
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  *cap = 0;
  const size_t n = std::max<size_t>(need, 1);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(ptr), n * sizeof(T));
  if (e == hipSuccess) *cap = n;
  return e;
}

template <class T>
hipError_t grow_pinned(T** ptr, size_t* cap, size_t need) {
  if (need <= *cap && *ptr) return hipSuccess;
  if (*ptr) (void)hipHostFree(*ptr);
  *ptr = nullptr;
  *cap = 0;
  const size_t n = std::max<size_t>(need, 1);
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(ptr), n * sizeof(T), hipHostMallocDefault);
  if (e == hipSuccess) *cap = n;
  return e;
}

int hip_fail(hipError_t e, const char* what) {
  return record_error(e == hipErrorOutOfMemory ? LP_ERR_NOMEM : LP_ERR_DEVICE,
                      std::string("reinversion: ") + what + ": " + hipGetErrorString(e));
}

int blas_fail(rocblas_status st, const char* what) {
  return record_error(st == rocblas_status_memory_error ? LP_ERR_NOMEM : LP_ERR_DEVICE,
                      std::string("reinversion: ") + what + ": " + rocblas_status_to_string(st));
}

#define R_HIP(expr, what)                          \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)
#define R_BLAS(expr, what)                                     \
  do {                                                         \
    rocblas_status st_ = (expr);                               \
    if (st_ != rocblas_status_success) return blas_fail(st_, what); \
  } while (0)

template <int NT, int RPT, int JB>
hipError_t launch_panel_step(double* M, int k, int j0, int jb, int32_t* pairs, int32_t* rowperm, int32_t* info,
                             hipStream_t s) {
  hipLaunchKernelGGL((k_lu_panel<NT, RPT, JB>), dim3(1), dim3(NT), 0, s, M, k, k, j0, jb, pairs, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int ncols = k - jb + 1;
  const int grid = (ncols + kRowPanelWaves - 1) / kRowPanelWaves;
  hipLaunchKernelGGL(k_lu_rowpanel, dim3(grid), dim3(kRowPanelThreads), 0, s, M, k, k, j0, jb, (const int32_t*)pairs,
                     rowperm);
  return hipGetLastError();
}

}  // namespace

void reinv_free(ReinvState* st) {
  if (!st) return;
  if (st->blas) (void)rocblas_destroy_handle(st->blas);
  for (void* p : {(void*)st->G, (void*)st->X, (void*)st->C, (void*)st->part, (void*)st->idx, (void*)st->aux})
    if (p) (void)hipFree(p);
  if (st->h_idx) (void)hipHostFree(st->h_idx);
  if (st->h_basis) (void)hipHostFree(st->h_basis);
  delete st;
}

int reinvert(const DevLP& d, const double* b, ReinvState** state, hipStream_t s, int* k_out) {
  if (!*state) {
    *state = new (std::nothrow) ReinvState();
    if (!*state) return record_error(LP_ERR_NOMEM, "reinversion: host allocation failed");
  }
  ReinvState* st = *state;
  if (!st->blas) {
    R_BLAS(rocblas_create_handle(&st->blas), "creating the BLAS handle");
    R_BLAS(rocblas_set_atomics_mode(st->blas, rocblas_atomics_not_allowed), "configuring the BLAS handle");
  }
  R_BLAS(rocblas_set_stream(st->blas, s), "configuring the BLAS handle");
  const int m = d.m, n = d.n, ld = d.ld;

  // 1. The basis, and the index sets of the block form.
  R_HIP(grow_pinned(&st->h_basis, &st->h_basis_cap, (size_t)m), "allocating pinned memory");
  R_HIP(hipMemcpyAsync(st->h_basis, d.basis, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s), "reading the basis");
  R_HIP(hipStreamSynchronize(s), "reading the basis");
  std::vector<int32_t> slack_pos(m, -1);
  std::vector<int32_t> kcol, kpos;
  kcol.reserve(m);
  kpos.reserve(m);
  for (int p = 0; p < m; ++p) {
    const int v = st->h_basis[p];
    if (v < 0 || v >= n + m) return record_error(LP_ERR_DEVICE, "reinversion: corrupt basis");
    if (v < n) {
      kcol.push_back(v);
      kpos.push_back(p);
    } else {
      slack_pos[v - n] = p;
    }
  }
  const int k = (int)kcol.size();
  const size_t nidx = 2 * (size_t)k + 2 * (size_t)m + ld;
  R_HIP(grow_pinned(&st->h_idx, &st->h_idx_cap, nidx), "allocating pinned memory");
  int32_t* h_kcol = st->h_idx;
  int32_t* h_kpos = h_kcol + k;
  int32_t* h_rowlist = h_kpos + k;
  int32_t* h_rinfo = h_rowlist + m;
  int32_t* h_colmap = h_rinfo + m;
  std::copy(kcol.begin(), kcol.end(), h_kcol);
  std::copy(kpos.begin(), kpos.end(), h_kpos);
  for (int j = 0; j < ld; ++j) h_colmap[j] = -1;
  int nr = 0;
  for (int i = 0; i < m; ++i)
    if (slack_pos[i] < 0) {
      h_colmap[i] = nr;
      h_rowlist[nr++] = i;
    }
  if (nr != k) return record_error(LP_ERR_DEVICE, "reinversion: basis list is not a basis");
  int ns = 0;
  for (int i = 0; i < m; ++i)
    if (slack_pos[i] >= 0) {
      h_rinfo[slack_pos[i]] = -(ns + 1);
      h_rowlist[k + ns++] = i;
    }
  for (int b = 0; b < k; ++b) h_rinfo[h_kpos[b]] = b;

  R_HIP(grow(&st->idx, &st->idx_cap, nidx), "allocating work memory");
  R_HIP(grow(&st->aux, &st->aux_cap, (size_t)m + 2 * kPairs + 2), "allocating work memory");
  R_HIP(hipMemcpyAsync(st->idx, st->h_idx, sizeof(int32_t) * nidx, hipMemcpyHostToDevice, s), "uploading indices");
  const int32_t* kcol_d = st->idx;
  const int32_t* kpos_d = kcol_d + k;
  const int32_t* rowlist_d = kpos_d + k;
  const int32_t* rinfo_d = rowlist_d + m;
  const int32_t* colmap_d = rinfo_d + m;
  int32_t* rowperm = st->aux;
  int32_t* pairs = rowperm + m;
  int32_t* info = pairs + 2 * kPairs + 1;

  const size_t kk = (size_t)k * k;
  R_HIP(grow(&st->G, &st->G_cap, (size_t)k * m), "allocating work memory");
  R_HIP(grow(&st->X, &st->X_cap, kk), "allocating work memory");
  R_HIP(grow(&st->C, &st->C_cap, (size_t)k * (m - k)), "allocating work memory");
  const int nchunk = std::max(1, (k + kWChunk - 1) / kWChunk);
  R_HIP(grow(&st->part, &st->part_cap, (size_t)nchunk * ld), "allocating work memory");

  hipLaunchKernelGGL(k_reinv_setup, dim3(std::max(1, (k + 255) / 256)), dim3(256), 0, s, rowperm, k, info);
  R_HIP(hipGetLastError(), "launching setup");

  if (k > 0) {
    // 1. G = [B11^T | B21^T]
    hipLaunchKernelGGL(k_gather, dim3((m + 31) / 32, (k + 31) / 32), dim3(32, 8), 0, s, d.A, ld, kcol_d, rowlist_d,
                       k, m, st->G);
    R_HIP(hipGetLastError(), "launching the gather");
    // 2. LU of M = G[:, 0:k] (leading dimension k).
    double* Mx = st->G;
    const double one = 1.0, minus_one = -1.0, zero = 0.0;
    for (int j0 = 0; j0 < k;) {
      const int R = k - j0;
      int jb;
      hipError_t e;
      // Panel shapes that keep the rows in registers without spills; R <= LP_MAX_ROWS.
      if (R <= 1024) {
        jb = std::min(32, R);
        e = launch_panel_step<1024, 1, 32>(Mx, k, j0, jb, pairs, rowperm, info, s);
      } else if (R <= 2048) {
        jb = 8;
        e = launch_panel_step<1024, 2, 8>(Mx, k, j0, jb, pairs, rowperm, info, s);
      } else if (R <= 4096) {
        jb = 4;
        e = launch_panel_step<1024, 4, 4>(Mx, k, j0, jb, pairs, rowperm, info, s);
      } else {
        jb = 2;
        e = launch_panel_step<1024, 10, 2>(Mx, k, j0, jb, pairs, rowperm, info, s);
      }
      R_HIP(e, "launching a panel factorisation");
      const int rest = k - j0 - jb;
      if (rest > 0) {
        R_BLAS(rocblas_dgemm(st->blas, rocblas_operation_none, rocblas_operation_none, rest, rest, jb, &minus_one,
                             Mx + (size_t)(j0 + jb) + (size_t)j0 * k, k, Mx + (size_t)j0 + (size_t)(j0 + jb) * k, k,
                             &one, Mx + (size_t)(j0 + jb) + (size_t)(j0 + jb) * k, k),
               "trailing update");
      }
      j0 += jb;
    }
    // 3. X = U^-1 L^-1 P
    hipLaunchKernelGGL(k_perm_matrix, dim3((unsigned)std::min<size_t>(8192, (kk + 255) / 256)), dim3(256), 0, s,
                       st->X, k, (const int32_t*)rowperm);
    R_HIP(hipGetLastError(), "launching the permutation");
    R_BLAS(rocblas_dtrsm(st->blas, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                         rocblas_diagonal_unit, k, k, &one, Mx, k, st->X, k),
           "solving with L");
    R_BLAS(rocblas_dtrsm(st->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                         rocblas_diagonal_non_unit, k, k, &one, Mx, k, st->X, k),
           "solving with U");
    // 4. C^T = -X B21^T
    if (m > k)
      R_BLAS(rocblas_dgemm(st->blas, rocblas_operation_none, rocblas_operation_none, k, m - k, k, &minus_one, st->X,
                           k, st->G + kk, k, &zero, st->C, k),
             "forming -B21 B11^-1");
  }
  // 5. B^-1, x_B, W, z.
  {
    const size_t total = (size_t)m * ld;
    hipLaunchKernelGGL(k_reinv_scatter, dim3((unsigned)std::min<size_t>(16384, (total + 255) / 256)), dim3(256), 0,
                       s, d.Binv, m, ld, k, rinfo_d, colmap_d, rowlist_d + k, (const double*)st->X,
                       (const double*)st->C, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching the scatter");
    hipLaunchKernelGGL(k_reinv_xb, dim3((unsigned)std::min(4096, (m + 3) / 4)), dim3(256), 0, s, d.xB, m, k, rinfo_d,
                       rowlist_d, (const double*)st->X, (const double*)st->C, b, d.eps_z, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching x_B");
    hipLaunchKernelGGL(k_reinv_w_part, dim3((ld + 255) / 256, nchunk), dim3(256), 0, s, st->part, ld, k, colmap_d,
                       kcol_d, d.chat, (const double*)st->X, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching W");
    hipLaunchKernelGGL(k_reinv_w_sum, dim3((ld + 255) / 256), dim3(256), 0, s, d.W, (const double*)st->part, ld,
                       nchunk, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching W");
    hipLaunchKernelGGL(k_reinv_finish, dim3(1), dim3(1024), 0, s, d.ctrl, k, kcol_d, kpos_d, d.chat,
                       (const double*)d.xB, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching the finish");
  }
  if (k_out) *k_out = k;
  return LP_OK;
}

}  // namespace lpgpu
