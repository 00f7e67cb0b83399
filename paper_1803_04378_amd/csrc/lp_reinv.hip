// Reinversion of the basis in FP64 (gfx950).
//
// With the slacks of the rows in S basic, order the basis as (structural columns K,
// slack columns of S) and the rows as (R = rows whose slack is nonbasic, then S):
//     B = [ B11  0 ]      B^-1 = [  B11^-1        0 ]
//         [ B21  I ],            [ -B21 B11^-1    I ],
// with B11 = A'[R, K] (order k = |K| = |R|) and B21 = A'[S, K].  Only B11 is factorised:
//   1. gather G = [B11^T | B21^T] (k x m, column-major) from A';
//   2. LU with partial pivoting of M = B11^T, blocked right-looking on two levels.  An
//      outer panel of kOuter columns is factorised by narrow inner panels: each inner
//      panel by one workgroup holding it in registers (the pivot search is a chain of
//      dependent reductions, so it stays inside one workgroup), then a second kernel
//      applies its row interchanges and U12 = L11^-1 A12 within the outer panel, and a
//      DGEMM updates the rest of the outer panel.  The outer panel's interchanges are
//      then applied to the columns outside it at once, U12 of the outer panel is a
//      triangular solve, and the trailing update A22 -= L21 U12 one DGEMM of depth
//      kOuter, so the trailing matrix is streamed once per kOuter columns;
//   3. X = M^-1 = U^-1 L^-1 P (two triangular solves on X = P), so that row b of B11^-1
//      is column b of X, contiguous;
//   4. C^T = -X B21^T (DGEMM): row s of -B21 B11^-1 is column s of C^T;
//   5. B^-1 written row by row in its row-major layout, x_B = B^-1 b, W = chat_B^T B^-1
//      and z = chat_B^T x_B from X and C^T.
// The DGEMMs and triangular solves are rocBLAS calls on the handle's stream (atomics off,
// so results are reproducible); everything else is below.
//
// Small blocks (k <= kSmallK, the common case: the optimal bases of the dense law hold a
// few hundred structural columns at most) take a shorter path with no library call: one
// workgroup inverts B11^T in LDS by Gauss-Jordan elimination with partial pivoting, and
// the rows -B21 B11^-1 are formed inside the kernel that writes B^-1.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "lp_reinv.h"
#include "lp_wave.h"
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
  int32_t* idx = nullptr;  // kcol (k) | kpos (k) | rowlist (m) | rinfo (m) | colmap (ld) | slack_pos (m)
  size_t idx_cap = 0;
  int32_t* aux = nullptr;  // rowperm (m) | opos (m) | inner list | outer list | info
  size_t aux_cap = 0;
  bool warmed = false;  // the large-block path has run once on this handle
};

namespace {

constexpr int kPairs = 64;        // row moves of one inner panel (at most 2 * 16 rows), room to spare
constexpr int kOuter = 128;       // outer panel width
constexpr int kOuterPairs = 2 * kOuter;
constexpr int kRowPanelThreads = 256;
constexpr int kWChunk = 64;  // b-range of one partial sum of W

// G[b + a*k] = A'[rowlist[a], kcol[b]] for b < k, a < m, through a 32 x 32 LDS tile so that
// both the reads (down a column of A') and the writes (down a column of G) coalesce.
__global__ void k_gather(const double* __restrict__ A, int ld, const int32_t* __restrict__ kcol,
                         const int32_t* __restrict__ rowlist, int k, int m, double* __restrict__ G,
                         const int32_t* __restrict__ info) {
  if (*info) return;  // the index sets are not valid
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

__global__ void k_reinv_setup(int32_t* rowperm, int32_t* opos, int k, int32_t* info) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) {
    rowperm[i] = i;
    opos[i] = i;
  }
  if (i == 0) *info = 0;
}

// Exclusive prefix count of a flag over a workgroup of kIndexBlock threads (ballots per
// wavefront, then the wavefront totals); `total` is the workgroup's count.
constexpr int kIndexBlock = 1024;
__device__ __forceinline__ int block_prefix_count(bool f, int* s_wsum, int& total) {
  constexpr int W = kIndexBlock / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long bal = __ballot(f);
  const int in_wave = __popcll(bal & ((1ull << lane) - 1ull));
  __syncthreads();  // s_wsum of the previous call has been read
  if (lane == 0) s_wsum[wave] = __popcll(bal);
  __syncthreads();
  int before = 0;
  total = 0;
  for (int w = 0; w < W; ++w) {
    const int c = s_wsum[w];
    before += w < wave ? c : 0;
    total += c;
  }
  return before + in_wave;
}

// The index sets of the block form from the basis list, on the device (one workgroup; m
// in chunks of kIndexBlock): K = basis positions holding a structural column, in position
// order, with kcol/kpos and rinfo[p] = its index b; R = rows whose slack is nonbasic,
// ascending, in rowlist[0..k) with colmap[i] = their index (-1 for every other column up
// to ld); S = the other rows, ascending, in rowlist[k..m), and rinfo[p] = -(s + 1) at the
// position p of the slack of the s-th of them.  A basis entry out of range, or a count of
// structural columns or of rows in R other than k, sets *info = 2 (nothing after this
// kernel then uses the index sets).
__global__ __launch_bounds__(kIndexBlock) void k_reinv_index(const int32_t* __restrict__ basis, int m, int n, int ld,
                                                            int k, int32_t* __restrict__ kcol,
                                                            int32_t* __restrict__ kpos, int32_t* __restrict__ rowlist,
                                                            int32_t* __restrict__ rinfo,
                                                            int32_t* __restrict__ colmap,
                                                            int32_t* __restrict__ slack_pos,
                                                            int32_t* __restrict__ info) {
  constexpr int B = kIndexBlock;
  __shared__ int s_wsum[B / 64];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  if (tid == 0) s_bad = 0;
  for (int i = tid; i < m; i += B) slack_pos[i] = -1;
  for (int j = tid; j < ld; j += B) colmap[j] = -1;
  __syncthreads();
  int nk = 0;
  for (int p0 = 0; p0 < m; p0 += B) {
    const int p = p0 + tid;
    const int v = p < m ? basis[p] : -1;
    const bool ok = p < m && v >= 0 && v < n + m;
    if (p < m && !ok) s_bad = 1;
    const bool isK = ok && v < n;
    if (ok && v >= n) slack_pos[v - n] = p;
    int tot;
    const int b = nk + block_prefix_count(isK, s_wsum, tot);
    if (isK && b < k) {
      kcol[b] = v;
      kpos[b] = p;
      rinfo[p] = b;
    }
    nk += tot;
  }
  __syncthreads();  // slack_pos is complete
  int nr = 0, ns = 0;
  for (int i0 = 0; i0 < m; i0 += B) {
    const int i = i0 + tid;
    const int sp = i < m ? slack_pos[i] : 0;
    const bool isR = i < m && sp < 0;
    int totR;
    const int rl = block_prefix_count(isR, s_wsum, totR);
    const int r = nr + rl;
    const int sidx = ns + (tid - rl);  // the chunk's valid rows are contiguous from tid 0
    if (isR && r < k) {
      colmap[i] = r;
      rowlist[r] = i;
    }
    if (i < m && !isR && k + sidx < m) {
      rowlist[k + sidx] = i;
      rinfo[sp] = -(sidx + 1);
    }
    nr += totR;
    ns += min(B, m - i0) - totR;
  }
  if (tid == 0 && (s_bad || nk != k || nr != k)) *info = 2;
}

// Factorises the panel M[j0:k, j0:j0+jb] in place (jb <= JB) with partial pivoting.
// Thread t of NT holds rows t, t + NT, ... (relative to j0) in registers, and rows stay
// where they are during the elimination: at column c the pivot is the not yet chosen row
// of largest |value| (lowest row on ties), its remaining entries are broadcast through
// LDS, and every other unchosen row is eliminated.  Each row keeps its unprocessed
// columns in a[] and its finished entries (multipliers, or its U row once chosen) in h[],
// both shifted by one position per column so that every register index is static and
// the column loop stays compact.  At the end the rows are written to their final places
// (the c-th pivot row to row c of the panel; rows displaced from the top to the places the
// pivot rows left), and the moves are listed as (dst, src) pairs for k_lu_rowpanel.  A
// zero pivot column sets *info.
template <int NT, int RPT, int JB>
__global__ __launch_bounds__(NT) void k_lu_panel(double* __restrict__ M, int ld, int k, int j0, int jb,
                                                 int32_t* __restrict__ pairs, int32_t* __restrict__ info) {
  constexpr int W = NT / 64;
  __shared__ double s_u[JB];
  __shared__ double red_v[2][W];  // alternate between columns: no barrier at a column's end
  __shared__ int red_i[2][W];
  __shared__ int s_piv[JB];
  __shared__ int s_dst[2 * JB], s_src[2 * JB];
  __shared__ int s_np;
  const int R = k - j0, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double a[RPT][JB], h[RPT][JB];
  bool done[RPT];
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int rho = tid + s * NT;
    done[s] = rho >= R;
#pragma unroll
    for (int c = 0; c < JB; ++c) {
      a[s][c] = (rho < R && c < jb) ? M[(size_t)(j0 + rho) + (size_t)(j0 + c) * ld] : 0.0;
      h[s][c] = 0.0;
    }
  }
  bool singular = false;
  for (int c = 0; c < jb; ++c) {
    const int bf = c & 1;
    // Pivot: largest |value| among unchosen rows, lowest row on ties, i.e. the
    // lexicographic minimum of (-|value|, row); 1.0 stands for "no candidate".
    double nv = 1.0;
    int bi = INT_MAX;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      double v = fabs(a[s][0]);
      v = v == v ? v : 0.0;  // a NaN never wins (and signals a singular block below)
      const bool take = !done[s] && -v < nv;
      nv = take ? -v : nv;
      bi = take ? tid + s * NT : bi;
    }
    detail::wave_lexmin(nv, bi);
    if (lane == 0) {
      red_v[bf][wave] = nv;
      red_i[bf][wave] = bi;
    }
    __syncthreads();
    nv = red_v[bf][0];
    bi = red_i[bf][0];
#pragma unroll
    for (int w = 1; w < W; ++w) {
      const double ov = red_v[bf][w];
      const int oi = red_i[bf][w];
      const bool take = detail::lex_less(ov, oi, nv, bi);
      nv = take ? ov : nv;
      bi = take ? oi : bi;
    }
    const double bv = -nv;
    if (!(bv > 0.0)) singular = true;
    const int p = bi;  // an unchosen row always exists: R - c >= 1
    // Selects rather than branches on the owning slot keep the register rows from being
    // copied at branch joins.
    {
      double uv[JB];
#pragma unroll
      for (int i = 0; i < JB; ++i) uv[i] = 0.0;
      bool mine = false;
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const bool hit = tid + s * NT == p;
#pragma unroll
        for (int i = 0; i < JB; ++i) uv[i] = hit ? a[s][i] : uv[i];
        done[s] = done[s] || hit;
        mine = mine || hit;
      }
      if (mine) {
#pragma unroll
        for (int i = 0; i < JB; ++i) s_u[i] = uv[i];
      }
    }
    if (tid == 0) s_piv[c] = p;
    __syncthreads();
    const double rpiv = 1.0 / s_u[0];  // one reciprocal per pivot, as LAPACK's unblocked LU
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const bool elim = !done[s];
      const double l = elim ? a[s][0] * rpiv : a[s][0];
#pragma unroll
      for (int i = 1; i < JB; ++i) {
        const double upd = fma(-l, s_u[i], a[s][i]);
        a[s][i] = elim ? upd : a[s][i];
      }
#pragma unroll
      for (int i = 0; i + 1 < JB; ++i) {
        a[s][i] = a[s][i + 1];
        h[s][i] = h[s][i + 1];
      }
      a[s][JB - 1] = 0.0;
      h[s][JB - 1] = l;
    }
    // No barrier here: the next column's pivot row is published only after its first
    // barrier, which every thread reaches after reading this column's row.
  }
  // Align the history so that h[c] holds column c (a narrower last panel shifted jb times).
  for (int x = jb; x < JB; ++x) {
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
#pragma unroll
      for (int i = 0; i + 1 < JB; ++i) h[s][i] = h[s][i + 1];
      h[s][JB - 1] = 0.0;
    }
  }
  // Final places: position c receives pivot row p_c; the rows of the top jb that were not
  // chosen fill, in ascending order, the places of the chosen rows from below the top.
  if (tid == 0) {
    int np = 0;
    bool top_chosen[JB];
#pragma unroll
    for (int i = 0; i < JB; ++i) top_chosen[i] = false;
    for (int c = 0; c < jb; ++c) {
      const int pc = s_piv[c];
#pragma unroll
      for (int i = 0; i < JB; ++i)
        if (i == pc) top_chosen[i] = true;
      if (pc != c) {
        s_dst[np] = c;
        s_src[np] = pc;
        ++np;
      }
    }
    int cv = 0;
#pragma unroll
    for (int i = 0; i < JB; ++i) {
      if (i >= jb || top_chosen[i]) continue;
      while (cv < jb && s_piv[cv] < jb) ++cv;  // next chosen row from below the top
      if (cv >= jb) break;  // cannot happen: as many such rows as unchosen top rows
      s_dst[np] = s_piv[cv];
      s_src[np] = i;
      ++np;
      ++cv;
    }
    s_np = np;
  }
  __syncthreads();
  const int np = s_np;
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int rho = tid + s * NT;
    if (rho >= R) continue;
    int dst = rho;
    for (int q = 0; q < np; ++q)
      if (s_src[q] == rho) dst = s_dst[q];
#pragma unroll
    for (int c = 0; c < JB; ++c)
      if (c < jb) M[(size_t)(j0 + dst) + (size_t)(j0 + c) * ld] = h[s][c];
  }
  if (tid < np) {
    pairs[tid] = j0 + s_dst[tid];
    pairs[kPairs + tid] = j0 + s_src[tid];
  }
  if (tid == 0) {
    pairs[2 * kPairs] = np;
    if (singular) *info = 1;
  }
}

// A row permutation given as (dst, src) pairs (row dst receives the row that was at src;
// np <= 4 * 64 pairs) applied to the columns c in [c_lo, c_hi) outside [skip_lo, skip_hi)
// and to the integer vector perm (the extra last "column"), then, for the columns from
// u_lo on, U12 = L11^-1 A12 by forward substitution with the unit lower L11 =
// M[j0:j0+jb, j0:j0+jb] (jb <= 32, staged in LDS).  One wavefront per column: lane q moves
// pairs q, q + 64, ..., and lane r holds row j0 + r during the substitution.
constexpr int kRowPanelWaves = kRowPanelThreads / 64;

__global__ __launch_bounds__(kRowPanelThreads) void k_lu_rowpanel(double* __restrict__ M, int ld, int c_lo, int c_hi,
                                                                  int skip_lo, int skip_hi, int u_lo, int j0, int jb,
                                                                  const int32_t* __restrict__ pairs, int cap,
                                                                  int32_t* __restrict__ perm) {
  __shared__ double s_l[32 * 32];
  const int np = pairs[2 * cap];
  if (u_lo < c_hi) {
    for (int e = threadIdx.x; e < 32 * 32; e += kRowPanelThreads) {
      const int r = e / 32, c = e % 32;
      s_l[e] = (c < r && r < jb) ? M[(size_t)(j0 + r) + (size_t)(j0 + c) * ld] : 0.0;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  int dst[4], src[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = lane + 64 * u;
    dst[u] = q < np ? pairs[q] : 0;
    src[u] = q < np ? pairs[cap + q] : 0;
  }
  const int nskip = skip_hi - skip_lo;
  const int ncols = c_hi - c_lo - nskip + 1;
  const int gw = blockIdx.x * kRowPanelWaves + (threadIdx.x >> 6);
  const int nw = gridDim.x * kRowPanelWaves;
  for (int e = gw; e < ncols; e += nw) {
    if (e == ncols - 1) {
      int v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (lane + 64 * u < np) v[u] = perm[src[u]];
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (lane + 64 * u < np) perm[dst[u]] = v[u];
      continue;
    }
    int col = c_lo + e;
    if (col >= skip_lo) col += nskip;
    double* colp = M + (size_t)col * ld;
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (lane + 64 * u < np) v[u] = colp[src[u]];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (lane + 64 * u < np) colp[dst[u]] = v[u];
    if (col >= u_lo) {
      // Reads after this wave's own writes above: same wavefront, program order.
      double x = lane < jb ? colp[j0 + lane] : 0.0;
      for (int c = 0; c + 1 < jb; ++c) {
        const double xc = __shfl(x, c);
        if (lane > c && lane < jb) x = fma(-s_l[lane * 32 + c], xc, x);
      }
      if (lane < jb) colp[j0 + lane] = x;
    }
  }
}

// U12 = L11^-1 A12 in place, for the unit lower triangular L11 = M[J0:J0+nb, J0:J0+nb]
// (nb <= kOuter) and A12 = M[J0:J0+nb, c0:c0+ncol], column-major with leading dimension
// ld.  Every workgroup stages L11 in LDS; each wavefront solves whole columns by forward
// substitution, lane l holding rows l and l + 64, the solved entry broadcast by readlane.
constexpr int kTrsmThreads = 256;
__device__ __forceinline__ double read_lane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__global__ __launch_bounds__(kTrsmThreads) void k_trsm_outer(double* __restrict__ M, int ld, int J0, int nb, int c0,
                                                           int ncol) {
  __shared__ double sL[kOuter * kOuter];  // column-major nb x nb
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int waves = kTrsmThreads / 64;
  for (int e = tid; e < nb * nb; e += kTrsmThreads) sL[e] = M[(size_t)(J0 + e % nb) + (size_t)(J0 + e / nb) * ld];
  __syncthreads();
  for (int col = blockIdx.x * waves + wave; col < ncol; col += gridDim.x * waves) {
    double* bcol = M + (size_t)J0 + (size_t)(c0 + col) * ld;
    const int i0 = lane, i1 = lane + 64;
    double b0 = i0 < nb ? bcol[i0] : 0.0;
    double b1 = i1 < nb ? bcol[i1] : 0.0;
    for (int j = 0; j < nb; ++j) {
      const double xj = j < 64 ? read_lane_d(b0, j) : read_lane_d(b1, j - 64);
      const double l0 = i0 > j && i0 < nb ? sL[i0 + j * nb] : 0.0;
      const double l1 = i1 > j && i1 < nb ? sL[i1 + j * nb] : 0.0;
      b0 = fma(-l0, xj, b0);
      b1 = fma(-l1, xj, b1);
    }
    if (i0 < nb) bcol[i0] = b0;
    if (i1 < nb) bcol[i1] = b1;
  }
}


// Composed interchanges of an outer panel: rows x in [r_lo, r_hi) whose opos[x] != x
// (opos[x] = row, at the start of the outer panel, of what is now row x) become pairs
// (x, opos[x]), and opos is reset to the identity for the next outer panel.
__global__ __launch_bounds__(1024) void k_lu_outer_pairs(int32_t* __restrict__ opos, int r_lo, int r_hi,
                                                         int32_t* __restrict__ pairs) {
  __shared__ int s_np;
  if (threadIdx.x == 0) s_np = 0;
  __syncthreads();
  for (int x = r_lo + threadIdx.x; x < r_hi; x += 1024) {
    const int o = opos[x];
    if (o != x) {
      const int q = atomicAdd(&s_np, 1);
      pairs[q] = x;
      pairs[kOuterPairs + q] = o;
      opos[x] = x;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) pairs[2 * kOuterPairs] = s_np;
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
// Writes B^-1 row by row: every column (ncols < 0), or only the ncols columns listed in
// cols (the list D: every other column is already exactly the unit vector it must be).
__global__ void k_reinv_scatter(double* __restrict__ Binv, int m, int ld, int k, const int32_t* __restrict__ rinfo,
                                const int32_t* __restrict__ colmap, const int32_t* __restrict__ srow,
                                const double* __restrict__ X, const double* __restrict__ Ct,
                                const int32_t* __restrict__ cols, int ncols, const int32_t* __restrict__ info) {
  if (*info) return;
  const bool all = ncols < 0;
  const int w = all ? ld : ncols;
  const size_t total = (size_t)m * w;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += stride) {
    const int p = (int)(e / w), t = (int)(e % w);
    const int j = all ? t : cols[t];
    const int a = colmap[j];
    const int ri = rinfo[p];
    double v;
    if (ri >= 0) {
      v = a >= 0 ? X[(size_t)a + (size_t)ri * k] : 0.0;
    } else {
      const int s = -ri - 1;
      v = a >= 0 ? Ct[(size_t)a + (size_t)s * k] : (j == srow[s] ? 1.0 : 0.0);
    }
    Binv[(size_t)p * ld + j] = v;
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

// The result goes to the copy of W that is current once no pivot is pending.
__global__ void k_reinv_w_sum(double* __restrict__ W0, double* __restrict__ W1, const Ctrl* __restrict__ ctl,
                              const double* __restrict__ part, int ld, int nchunk, const int32_t* __restrict__ info) {
  if (*info) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ld) return;
  double* W = ctl->wcur ? W1 : W0;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += part[(size_t)c * ld + j];
  W[j] = acc;
}

// z = chat_B^T x_B over the structural basic variables, then the control block: the new
// B^-1 already reflects the last pivot, so no row update is pending any more.
// Also resets the list D of columns of B^-1 that may differ from unit vectors to the
// columns of the rows whose slack is nonbasic (rowlist[0..k)): after the reinversion every
// other column is exactly a unit vector.
__global__ __launch_bounds__(1024) void k_reinv_finish(Ctrl* ctl, int m, int k, const int32_t* __restrict__ kcol,
                                                       const int32_t* __restrict__ kpos,
                                                       const int32_t* __restrict__ rowlist,
                                                       const int32_t* __restrict__ colmap,
                                                       int32_t* __restrict__ dlist, int32_t* __restrict__ inD,
                                                       const double* __restrict__ chat,
                                                       const double* __restrict__ xB,
                                                       const int32_t* __restrict__ info) {
  __shared__ double red[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (*info == 0) {
    for (int j = tid; j < m; j += 1024) inD[j] = colmap[j] >= 0 ? 1 : 0;
    for (int a = tid; a < k; a += 1024) dlist[a] = rowlist[a];
  }
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
      ctl->nD = k;
      ctl->n_reinv += 1;
    } else {
      ctl->n_reinv_failed += 1;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Small blocks.
constexpr int kSmallK = 128;

// X = M^-1 for M = G[:, 0:k] (column-major, k <= kSmallK) by in-place Gauss-Jordan
// elimination with partial pivoting, one workgroup.  Thread 8j + g holds column j of rows
// g, g + 8, ... (at most 16) in registers, so the eight holders of a column are adjacent
// lanes of one wavefront.  Column c: its holders find the row of largest |value| at or
// below the diagonal (lowest row on ties) with three shuffles and publish the old column c;
// after a barrier the holders of rows p and c publish those rows; after a second barrier
// row c becomes row p scaled by the reciprocal pivot with its diagonal entry replaced by
// that reciprocal, row p becomes the old row c, and column c is eliminated from every
// other row.  The LDS buffers alternate between columns.  The row exchanges make the
// result (P M)^-1 = M^-1 P^T, so its column c is column idx[c] of M^-1.
// KMAX (<= kSmallK) bounds k; the workgroup has 8 * KMAX threads, so that smaller blocks
// synchronise fewer wavefronts per column.
template <int KMAX>
__global__ __launch_bounds__(8 * KMAX) void k_gj_inverse(const double* __restrict__ G, int k,
                                                         double* __restrict__ X, int32_t* __restrict__ info) {
  constexpr int kGJRows = KMAX / 8;  // rows of the block one thread holds
  __shared__ double s_row[2][KMAX], s_rowc[2][KMAX], s_col[2][KMAX];
  __shared__ double s_pv[2];
  __shared__ int s_p[2];
  __shared__ int s_idx[KMAX];
  __shared__ int s_sing;
  const int tid = threadIdx.x;
  const int grp = tid & 7, jcol = tid >> 3;
  const bool active = jcol < k;
  double a[kGJRows];
#pragma unroll
  for (int u = 0; u < kGJRows; ++u) {
    const int i = grp + 8 * u;
    a[u] = (active && i < k) ? G[(size_t)i + (size_t)jcol * k] : 0.0;
  }
  if (tid < k) s_idx[tid] = tid;
  if (tid == 0) s_sing = 0;
  __syncthreads();
  for (int c = 0; c < k; ++c) {
    const int bf = c & 1;
    if (jcol == c) {
      double bv = -1.0, sv = 0.0;
      int bi = INT_MAX;
#pragma unroll
      for (int u = 0; u < kGJRows; ++u) {
        const int i = grp + 8 * u;
        if (i < k) {
          s_col[bf][i] = a[u];
          if (i >= c) {
            double v = fabs(a[u]);
            v = v == v ? v : 0.0;
            if (v > bv) {
              bv = v;
              bi = i;
              sv = a[u];
            }
          }
        }
      }
#pragma unroll
      for (int off = 1; off < 8; off <<= 1) {
        const double ov = __shfl_xor(bv, off);
        const double osv = __shfl_xor(sv, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
          sv = osv;
        }
      }
      if (grp == 0) {
        s_p[bf] = bi;
        s_pv[bf] = sv;
        if (!(bv > 0.0)) s_sing = 1;
        if (bi != c) {
          const int t = s_idx[c];
          s_idx[c] = s_idx[bi];
          s_idx[bi] = t;
        }
      }
    }
    __syncthreads();
    const int p = s_p[bf];
    // Branch-free from here on (selects only), so that the register rows are never
    // copied at branch joins.
    if (active) {
      double vp = 0.0, vc = 0.0;
#pragma unroll
      for (int u = 0; u < kGJRows; ++u) {
        const int i = grp + 8 * u;
        vp = i == p ? a[u] : vp;
        vc = i == c ? a[u] : vc;
      }
      if ((p & 7) == grp) s_row[bf][jcol] = vp;
      if ((c & 7) == grp) s_rowc[bf][jcol] = vc;
    }
    __syncthreads();
    if (active) {
      const double pivinv = 1.0 / s_pv[bf];
      const double rowc = (jcol == c ? 1.0 : s_row[bf][jcol]) * pivinv;
      const double oldc = s_rowc[bf][jcol];
      const double colc = s_col[bf][c];
      const bool on_c = jcol == c;
#pragma unroll
      for (int u = 0; u < kGJRows; ++u) {
        const int i = grp + 8 * u;
        const bool isp = i == p;
        const double f = isp ? colc : s_col[bf][i < k ? i : 0];
        const double base = on_c ? 0.0 : (isp ? oldc : a[u]);
        const double upd = fma(-f, rowc, base);
        a[u] = i < k ? (i == c ? rowc : upd) : a[u];
      }
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int u = 0; u < kGJRows; ++u) {
      const int i = grp + 8 * u;
      if (i < k) X[(size_t)i + (size_t)s_idx[jcol] * k] = a[u];
    }
  }
  if (tid == 0 && s_sing) *info = 1;
}

// B^-1 in its m x ld row-major layout, 4 rows per workgroup.  A structural basis position
// b copies column b of X; a slack position s forms -sum_b B21[s, b] B11^-1[b, :] from the
// column k + s of G and X (4 rows share each read of X).  Every column is written
// (ncols < 0) or only the ncols columns listed in cols, as k_reinv_scatter.
constexpr int kScatterRows = 4;

__global__ __launch_bounds__(256) void k_reinv_scatter_small(double* __restrict__ Binv, int m, int ld, int k,
                                                              const int32_t* __restrict__ rinfo,
                                                              const int32_t* __restrict__ colmap,
                                                              const int32_t* __restrict__ srow,
                                                              const double* __restrict__ X,
                                                              const double* __restrict__ G,
                                                              const int32_t* __restrict__ cols, int ncols,
                                                              const int32_t* __restrict__ info) {
  if (*info) return;
  __shared__ double s_g[kScatterRows][kSmallK];
  __shared__ double s_v[kScatterRows][kSmallK];
  const int p0 = blockIdx.x * kScatterRows, tid = threadIdx.x;
  int ri[kScatterRows];
#pragma unroll
  for (int r = 0; r < kScatterRows; ++r) {
    ri[r] = p0 + r < m ? rinfo[p0 + r] : 0;
    for (int b = tid; b < k; b += 256)
      s_g[r][b] = (p0 + r < m && ri[r] < 0) ? G[(size_t)b + (size_t)(k + (-ri[r] - 1)) * k] : 0.0;
  }
  __syncthreads();
  if (tid < k) {
    const int a = tid;
    double acc[kScatterRows];
#pragma unroll
    for (int r = 0; r < kScatterRows; ++r) acc[r] = 0.0;
    for (int b = 0; b < k; ++b) {
      const double x = X[(size_t)a + (size_t)b * k];
#pragma unroll
      for (int r = 0; r < kScatterRows; ++r) acc[r] = fma(s_g[r][b], x, acc[r]);
    }
#pragma unroll
    for (int r = 0; r < kScatterRows; ++r)
      s_v[r][a] = ri[r] >= 0 ? X[(size_t)a + (size_t)ri[r] * k] : -acc[r];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kScatterRows; ++r) {
    const int p = p0 + r;
    if (p >= m) break;
    const int sr = ri[r] < 0 ? srow[-ri[r] - 1] : -1;
    double* row = Binv + (size_t)p * ld;
    const bool all = ncols < 0;
    const int w = all ? ld : ncols;
    for (int t = tid; t < w; t += 256) {
      const int j = all ? t : cols[t];
      const int a = colmap[j];
      row[j] = a >= 0 ? s_v[r][a] : (j == sr ? 1.0 : 0.0);
    }
  }
}

// x_B of the structural basis positions, x_K = B11^-1 b_R (column b of X dotted with b_R),
// also kept in xs for the slack positions.
__global__ __launch_bounds__(256) void k_reinv_xstruct(double* __restrict__ xB, double* __restrict__ xs, int k,
                                                       const int32_t* __restrict__ kpos,
                                                       const int32_t* __restrict__ rowlist,
                                                       const double* __restrict__ X, const double* __restrict__ b,
                                                       double eps_z, const int32_t* __restrict__ info) {
  if (*info) return;
  __shared__ double s_b[kSmallK];
  const int bb = threadIdx.x;
  if (bb < k) s_b[bb] = b[rowlist[bb]];
  __syncthreads();
  if (bb >= k) return;
  double acc = 0.0;
#pragma unroll 8
  for (int a = 0; a < k; ++a) acc = fma(X[(size_t)a + (size_t)bb * k], s_b[a], acc);
  xs[bb] = acc;
  xB[kpos[bb]] = fabs(acc) < eps_z ? 0.0 : acc;
}

// x_B of the slack basis positions: b_S - B21 x_K, one wavefront per position.
__global__ void k_reinv_xslack(double* __restrict__ xB, int m, int k, const int32_t* __restrict__ rinfo,
                               const int32_t* __restrict__ srow, const double* __restrict__ G,
                               const double* __restrict__ xs, const double* __restrict__ b, double eps_z,
                               const int32_t* __restrict__ info) {
  if (*info) return;
  const int lane = threadIdx.x & 63;
  const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nw = (gridDim.x * blockDim.x) >> 6;
  for (int p = gw; p < m; p += nw) {
    const int ri = rinfo[p];
    if (ri >= 0) continue;
    const int s = -ri - 1;
    const double* g = G + (size_t)(k + s) * k;
    double acc = 0.0;
    for (int bb = lane; bb < k; bb += 64) acc = fma(g[bb], xs[bb], acc);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) {
      const double x = b[srow[s]] - acc;
      xB[p] = fabs(x) < eps_z ? 0.0 : x;
    }
  }
}

// W_j = sum_b chat_{kcol[b]} B11^-1[b, a] for j = rowlist[a], 0 elsewhere, into the copy of
// W that is current once no pivot is pending.
__global__ void k_reinv_w_small(double* __restrict__ W0, double* __restrict__ W1, const Ctrl* __restrict__ ctl,
                                int ld, int k, const int32_t* __restrict__ colmap, const int32_t* __restrict__ kcol,
                                const double* __restrict__ chat, const double* __restrict__ X,
                                const int32_t* __restrict__ info) {
  if (*info) return;
  __shared__ double s_c[kSmallK];
  for (int bb = threadIdx.x; bb < k; bb += blockDim.x) s_c[bb] = chat[kcol[bb]];
  __syncthreads();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ld) return;
  const int a = colmap[j];
  double acc = 0.0;
  if (a >= 0) {
#pragma unroll 8
    for (int bb = 0; bb < k; ++bb) acc = fma(s_c[bb], X[(size_t)a + (size_t)bb * k], acc);
  }
  (ctl->wcur ? W1 : W0)[j] = acc;
}

// Grow-only device buffer; capacity at least doubles so that a basis block growing over a
// solve reallocates O(log) times (a free synchronises the device).
template <class T>
hipError_t grow(T** ptr, size_t* cap, size_t need, size_t limit) {
  if (need <= *cap && *ptr) return hipSuccess;
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  const size_t n = std::max<size_t>(std::max(need, std::min(2 * *cap, limit)), 1);
  *cap = 0;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(ptr), n * sizeof(T));
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

// Inner panel j0..j0+jb of the outer panel J0..J0+JBo: factorisation, then its row
// interchanges on the other columns of the outer panel (and on opos) with U12 for the
// columns right of it.
template <int NT, int RPT, int JB>
hipError_t launch_inner_panel(double* M, int k, int J0, int JBo, int j0, int jb, int32_t* pairs, int32_t* opos,
                              int32_t* info, hipStream_t s) {
  hipLaunchKernelGGL((k_lu_panel<NT, RPT, JB>), dim3(1), dim3(NT), 0, s, M, k, k, j0, jb, pairs, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int ncols = JBo - jb + 1;
  const int grid = (ncols + kRowPanelWaves - 1) / kRowPanelWaves;
  hipLaunchKernelGGL(k_lu_rowpanel, dim3(grid), dim3(kRowPanelThreads), 0, s, M, k, J0, J0 + JBo, j0, j0 + jb,
                     j0 + jb, j0, jb, (const int32_t*)pairs, kPairs, opos);
  return hipGetLastError();
}

}  // namespace

void reinv_free(ReinvState* st) {
  if (!st) return;
  if (st->blas) (void)rocblas_destroy_handle(st->blas);
  for (void* p : {(void*)st->G, (void*)st->X, (void*)st->C, (void*)st->part, (void*)st->idx, (void*)st->aux})
    if (p) (void)hipFree(p);
  delete st;
}

namespace {

// Steps 2-4 of the large-block path on st->G (k x m, k >= 1): LU of M = G[:, 0:k] in place,
// X = M^-1 = (B11^-1)^T, and C^T = -X B21^T when m > k.  A zero pivot column sets *info.
int invert_large(ReinvState* st, int k, int m, int32_t* rowperm, int32_t* opos, int32_t* pairs, int32_t* opairs,
                 int32_t* info, hipStream_t s) {
  const size_t kk = (size_t)k * k;
  // 2. LU of M = G[:, 0:k] (leading dimension k).
  double* Mx = st->G;
  const double one = 1.0, minus_one = -1.0, zero = 0.0;
  for (int J0 = 0; J0 < k; J0 += kOuter) {
    const int JBo = std::min(kOuter, k - J0);
    for (int j0 = J0; j0 < J0 + JBo;) {
      const int R = k - j0, room = J0 + JBo - j0;
      int jb;
      hipError_t e;
      // Inner panel shapes that keep the rows in registers without spills; R <= LP_MAX_ROWS.
      // The per-column cost is synchronisation across the workgroup's wavefronts, so the
      // workgroup is no larger than the panel needs.
      if (R <= 256) {
        jb = std::min(16, room);
        e = launch_inner_panel<256, 1, 16>(Mx, k, J0, JBo, j0, jb, pairs, opos, info, s);
      } else if (R <= 512) {
        jb = std::min(16, room);
        e = launch_inner_panel<512, 1, 16>(Mx, k, J0, JBo, j0, jb, pairs, opos, info, s);
      } else if (R <= 1024) {
        jb = std::min(16, room);
        e = launch_inner_panel<1024, 1, 16>(Mx, k, J0, JBo, j0, jb, pairs, opos, info, s);
      } else if (R <= 2048) {
        jb = std::min(8, room);
        e = launch_inner_panel<1024, 2, 8>(Mx, k, J0, JBo, j0, jb, pairs, opos, info, s);
      } else if (R <= 4096) {
        jb = std::min(4, room);
        e = launch_inner_panel<1024, 4, 4>(Mx, k, J0, JBo, j0, jb, pairs, opos, info, s);
      } else {
        jb = std::min(2, room);
        e = launch_inner_panel<1024, 10, 2>(Mx, k, J0, JBo, j0, jb, pairs, opos, info, s);
      }
      R_HIP(e, "launching a panel factorisation");
      const int rows = k - j0 - jb, cols = J0 + JBo - j0 - jb;
      if (rows > 0 && cols > 0)
        R_BLAS(rocblas_dgemm(st->blas, rocblas_operation_none, rocblas_operation_none, rows, cols, jb, &minus_one,
                             Mx + (size_t)(j0 + jb) + (size_t)j0 * k, k, Mx + (size_t)j0 + (size_t)(j0 + jb) * k, k,
                             &one, Mx + (size_t)(j0 + jb) + (size_t)(j0 + jb) * k, k),
               "inner update");
      j0 += jb;
    }
    // The outer panel's interchanges on the columns outside it and on rowperm.
    hipLaunchKernelGGL(k_lu_outer_pairs, dim3(1), dim3(1024), 0, s, opos, J0, k, opairs);
    R_HIP(hipGetLastError(), "launching the interchange list");
    {
      const int ncols = k - JBo + 1;
      hipLaunchKernelGGL(k_lu_rowpanel, dim3((ncols + kRowPanelWaves - 1) / kRowPanelWaves), dim3(kRowPanelThreads),
                         0, s, Mx, k, 0, k, J0, J0 + JBo, k, 0, 0, (const int32_t*)opairs, kOuterPairs, rowperm);
      R_HIP(hipGetLastError(), "launching the interchanges");
    }
    const int rest = k - J0 - JBo;
    if (rest > 0) {
      // (not rocBLAS: its choice of method varies with the width rest, and each method's
      // first use in a process stalls for tens of milliseconds)
      const int waves = kTrsmThreads / 64;
      hipLaunchKernelGGL(k_trsm_outer, dim3((rest + waves - 1) / waves), dim3(kTrsmThreads), 0, s, Mx, k, J0, JBo,
                         J0 + JBo, rest);
      R_HIP(hipGetLastError(), "launching the outer U12 solve");
      R_BLAS(rocblas_dgemm(st->blas, rocblas_operation_none, rocblas_operation_none, rest, rest, JBo, &minus_one,
                           Mx + (size_t)(J0 + JBo) + (size_t)J0 * k, k, Mx + (size_t)J0 + (size_t)(J0 + JBo) * k, k,
                           &one, Mx + (size_t)(J0 + JBo) + (size_t)(J0 + JBo) * k, k),
             "trailing update");
    }
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
  return LP_OK;
}

// A well-conditioned stand-in block (identity B11, B21 = 0) for the warm-up.
__global__ void k_warm_block(double* G, int k, int m) {
  const size_t total = (size_t)k * m;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x)
    G[e] = (e % k) == (e / k) ? 1.0 : 0.0;
}

constexpr int kWarmK = 160;  // larger than kSmallK, so that every large-path step runs

}  // namespace

int reinv_prepare(ReinvState** state, int m, int ld) {
  if (!*state) {
    *state = new (std::nothrow) ReinvState();
    if (!*state) return record_error(LP_ERR_NOMEM, "reinversion: host allocation failed");
  }
  ReinvState* st = *state;
  if (!st->blas) {
    // rocBLAS loads its kernels lazily on first use (tens of milliseconds); load them once
    // per process here, outside any solve.
    static std::once_flag loaded;
    std::call_once(loaded, [] { rocblas_initialize(); });
    R_BLAS(rocblas_create_handle(&st->blas), "creating the BLAS handle");
    R_BLAS(rocblas_set_atomics_mode(st->blas, rocblas_atomics_not_allowed), "configuring the BLAS handle");
  }
  // Work memory for blocks up to kSmallK allocated up front (no allocation, and so no
  // device synchronisation, inside a solve unless the block grows past that).
  const size_t mm = (size_t)m * m, ks = (size_t)std::min(m, kSmallK);
  R_HIP(grow(&st->idx, &st->idx_cap, 5 * (size_t)m + ld, 5 * (size_t)m + ld), "allocating work memory");
  const size_t naux = 2 * (size_t)m + 2 * kPairs + 2 * kOuterPairs + 3;
  R_HIP(grow(&st->aux, &st->aux_cap, naux, naux), "allocating work memory");
  R_HIP(grow(&st->G, &st->G_cap, ks * m, mm), "allocating work memory");
  R_HIP(grow(&st->X, &st->X_cap, ks * ks, mm), "allocating work memory");
  R_HIP(grow(&st->part, &st->part_cap, 2 * (size_t)ld, ((size_t)m / kWChunk + 1) * ld), "allocating work memory");
  if (!st->warmed && m > kSmallK) {
    // The first launch of a rocBLAS kernel loads its code object and the first triangular
    // solve of a handle sizes its workspace: 40-130 ms stalls observed in the middle of a
    // solve.  Run the large-block path once here on a stand-in block of order kWarmK, on
    // the null stream, outside any solve.
    const int kw = std::min(m, kWarmK);
    R_HIP(grow(&st->G, &st->G_cap, (size_t)kw * m, mm), "allocating work memory");
    R_HIP(grow(&st->X, &st->X_cap, (size_t)kw * kw, mm), "allocating work memory");
    if (m > kw) R_HIP(grow(&st->C, &st->C_cap, (size_t)kw * (m - kw), mm / 4 + 1), "allocating work memory");
    R_BLAS(rocblas_set_stream(st->blas, nullptr), "configuring the BLAS handle");
    int32_t* rowperm = st->aux;
    int32_t* opos = rowperm + m;
    int32_t* pairs = opos + m;
    int32_t* opairs = pairs + 2 * kPairs + 1;
    int32_t* info = opairs + 2 * kOuterPairs + 1;
    hipLaunchKernelGGL(k_warm_block, dim3(1024), dim3(256), 0, nullptr, st->G, kw, m);
    R_HIP(hipGetLastError(), "launching the warm-up block");
    hipLaunchKernelGGL(k_reinv_setup, dim3((kw + 255) / 256), dim3(256), 0, nullptr, rowperm, opos, kw, info);
    R_HIP(hipGetLastError(), "launching setup");
    const int rc = invert_large(st, kw, m, rowperm, opos, pairs, opairs, info, nullptr);
    if (rc != LP_OK) return rc;
    R_HIP(hipStreamSynchronize(nullptr), "warming up the factorisation");
    st->warmed = true;
  }
  return LP_OK;
}

int reinvert(const DevLP& d, const double* b, ReinvState** state, hipStream_t s, int k, int nd_old, int* k_out) {
  int rc = reinv_prepare(state, d.m, d.ld);
  if (rc != LP_OK) return rc;
  ReinvState* st = *state;
  const int m = d.m, n = d.n, ld = d.ld;
  if (k < 0 || k > m) return record_error(LP_ERR_DEVICE, "reinversion: structural count out of range");
  R_BLAS(rocblas_set_stream(st->blas, s), "configuring the BLAS handle");

  // 1. The index sets of the block form, built on the device from the basis list.
  const size_t nidx = 2 * (size_t)k + 3 * (size_t)m + ld;
  R_HIP(grow(&st->idx, &st->idx_cap, nidx, 5 * (size_t)m + ld), "allocating work memory");
  const size_t naux = 2 * (size_t)m + 2 * kPairs + 2 * kOuterPairs + 3;
  R_HIP(grow(&st->aux, &st->aux_cap, naux, naux), "allocating work memory");
  int32_t* kcol_d = st->idx;
  int32_t* kpos_d = kcol_d + k;
  int32_t* rowlist_d = kpos_d + k;
  int32_t* rinfo_d = rowlist_d + m;
  int32_t* colmap_d = rinfo_d + m;
  int32_t* slackpos_d = colmap_d + ld;
  int32_t* rowperm = st->aux;
  int32_t* opos = rowperm + m;
  int32_t* pairs = opos + m;
  int32_t* opairs = pairs + 2 * kPairs + 1;
  int32_t* info = opairs + 2 * kOuterPairs + 1;

  const size_t kk = (size_t)k * k, mm = (size_t)m * m;
  R_HIP(grow(&st->G, &st->G_cap, (size_t)k * m, mm), "allocating work memory");
  R_HIP(grow(&st->X, &st->X_cap, kk, mm), "allocating work memory");
  const bool small = k <= kSmallK;
  if (!small) R_HIP(grow(&st->C, &st->C_cap, (size_t)k * (m - k), mm / 4 + 1), "allocating work memory");
  const int nchunk = std::max(1, (k + kWChunk - 1) / kWChunk);
  R_HIP(grow(&st->part, &st->part_cap, std::max((size_t)nchunk * ld, (size_t)k), ((size_t)m / kWChunk + 1) * ld),
        "allocating work memory");
  // Columns of B^-1 to write: those of the list D, which holds every column that can
  // differ from a unit vector (the new R included), while it is short; else all.
  const int ncols = (nd_old >= 0 && (size_t)nd_old * 8 <= (size_t)ld) ? nd_old : -1;

  hipLaunchKernelGGL(k_reinv_setup, dim3(std::max(1, (k + 255) / 256)), dim3(256), 0, s, rowperm, opos, k, info);
  R_HIP(hipGetLastError(), "launching setup");
  hipLaunchKernelGGL(k_reinv_index, dim3(1), dim3(kIndexBlock), 0, s, (const int32_t*)d.basis, m, n, ld, k, kcol_d,
                     kpos_d, rowlist_d, rinfo_d, colmap_d, slackpos_d, info);
  R_HIP(hipGetLastError(), "launching the index sets");

  if (k > 0) {
    // 1. G = [B11^T | B21^T]
    hipLaunchKernelGGL(k_gather, dim3((m + 31) / 32, (k + 31) / 32), dim3(32, 8), 0, s, d.A, ld,
                       (const int32_t*)kcol_d, (const int32_t*)rowlist_d, k, m, st->G, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching the gather");
  }
  if (k > 0 && small) {
    // 2'-4'. X = M^-1 in one workgroup; -B21 B11^-1 is formed while writing B^-1.
    if (k <= 32)
      hipLaunchKernelGGL(k_gj_inverse<32>, dim3(1), dim3(8 * 32), 0, s, (const double*)st->G, k, st->X, info);
    else if (k <= 64)
      hipLaunchKernelGGL(k_gj_inverse<64>, dim3(1), dim3(8 * 64), 0, s, (const double*)st->G, k, st->X, info);
    else
      hipLaunchKernelGGL(k_gj_inverse<kSmallK>, dim3(1), dim3(8 * kSmallK), 0, s, (const double*)st->G, k, st->X,
                         info);
    R_HIP(hipGetLastError(), "launching the small inverse");
  } else if (k > 0) {
    if ((rc = invert_large(st, k, m, rowperm, opos, pairs, opairs, info, s)) != LP_OK) return rc;
  }
  // 5. B^-1, x_B, W, z.
  if (small) {
    hipLaunchKernelGGL(k_reinv_scatter_small, dim3((m + kScatterRows - 1) / kScatterRows), dim3(256), 0, s, d.Binv, m,
                       ld, k, rinfo_d, colmap_d, rowlist_d + k, (const double*)st->X, (const double*)st->G,
                       (const int32_t*)d.dlist, ncols, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching the scatter");
    hipLaunchKernelGGL(k_reinv_xstruct, dim3(1), dim3(kSmallK), 0, s, d.xB, st->part, k, kpos_d, rowlist_d,
                       (const double*)st->X, b, d.eps_z, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching x_B");
    hipLaunchKernelGGL(k_reinv_xslack, dim3((unsigned)std::min(4096, (m + 3) / 4)), dim3(256), 0, s, d.xB, m, k,
                       rinfo_d, rowlist_d + k, (const double*)st->G, (const double*)st->part, b, d.eps_z,
                       (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching x_B");
    hipLaunchKernelGGL(k_reinv_w_small, dim3((ld + 255) / 256), dim3(256), 0, s, d.W0, d.W1, (const Ctrl*)d.ctrl, ld,
                       k, colmap_d, kcol_d, d.chat, (const double*)st->X, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching W");
    hipLaunchKernelGGL(k_reinv_finish, dim3(1), dim3(1024), 0, s, d.ctrl, m, k, kcol_d, kpos_d, rowlist_d, colmap_d,
                       d.dlist, d.inD, d.chat, (const double*)d.xB, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching the finish");
  } else {
    const size_t total = (size_t)m * (ncols < 0 ? ld : ncols);
    hipLaunchKernelGGL(k_reinv_scatter, dim3((unsigned)std::min<size_t>(16384, (total + 255) / 256)), dim3(256), 0,
                       s, d.Binv, m, ld, k, rinfo_d, colmap_d, rowlist_d + k, (const double*)st->X,
                       (const double*)st->C, (const int32_t*)d.dlist, ncols, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching the scatter");
    hipLaunchKernelGGL(k_reinv_xb, dim3((unsigned)std::min(4096, (m + 3) / 4)), dim3(256), 0, s, d.xB, m, k, rinfo_d,
                       rowlist_d, (const double*)st->X, (const double*)st->C, b, d.eps_z, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching x_B");
    hipLaunchKernelGGL(k_reinv_w_part, dim3((ld + 255) / 256, nchunk), dim3(256), 0, s, st->part, ld, k, colmap_d,
                       kcol_d, d.chat, (const double*)st->X, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching W");
    hipLaunchKernelGGL(k_reinv_w_sum, dim3((ld + 255) / 256), dim3(256), 0, s, d.W0, d.W1, (const Ctrl*)d.ctrl,
                       (const double*)st->part, ld, nchunk, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching W");
    hipLaunchKernelGGL(k_reinv_finish, dim3(1), dim3(1024), 0, s, d.ctrl, m, k, kcol_d, kpos_d, rowlist_d, colmap_d,
                       d.dlist, d.inD, d.chat, (const double*)d.xB, (const int32_t*)info);
    R_HIP(hipGetLastError(), "launching the finish");
  }
  if (k_out) *k_out = k;
  return LP_OK;
}

}  // namespace lpgpu
