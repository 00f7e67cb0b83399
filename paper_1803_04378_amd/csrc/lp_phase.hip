// Two-phase start (Section 3.4, finding the initial feasible solution, by the textbook
// two-phase method it cites): the kernels of the switch from phase 1 to phase 2.
//
// Phase 1 runs on the iteration kernels unchanged, with the artificial variables (the
// unit columns of the rows that have no basic slack) costed 1 and every other column 0.
// When it prices out optimal, the host:
//   - declares the LP infeasible if the phase-1 objective exceeds its tolerance, else
//   - for each row, in ascending order, whose basic variable is still artificial (at zero
//     level), replaces that variable by the nonbasic, non-barred column with the largest
//     |entry| in the row's line of the tableau, B^-1[r,:] a_j, through a pivot with step
//     0; a row with no entry above eps_p is redundant and keeps its artificial variable;
//   - restores the LP's own costs and recomputes W = chat_B^T B^-1 and z = chat_B^T x_B
//     from their definitions; the iteration then continues as phase 2.
// None of these kernels runs inside the iteration graph, and none runs with a pivot
// pending, so the FTRAN buffer alpha0 and the pivot-row buffer rho are free scratch.
// Each sum is an ascending fma chain over one thread, the order their definitions are
// written in: given the same tableau, the switch is bit for bit the plain definition.
// These are one-off passes (one per artificial variable left in the basis, plus one
// re-pricing), far from the per-iteration cost, so they favour that exactness over speed.
#include <algorithm>

#include "lp_device.h"
#include "lp_wave.h"

namespace lpgpu {
namespace {

using namespace detail;

constexpr int kPhaseBlock = 256;
constexpr int kZBlock = 1024;

// W_j = sum_i chat_{basis[i]} B^-1[i, j] over the rows whose basic variable has a nonzero
// cost, ascending i, for every j < ld (the zero padding stays zero); stored in both copies
// of W.  The costs of a chunk of rows are staged in LDS; thread j walks column j.
__global__ __launch_bounds__(kPhaseBlock) void k_reprice_w(DevLP lp) {
  __shared__ double s_cb[kPhaseBlock];
  const int m = lp.m, ld = lp.ld;
  const int j = blockIdx.x * kPhaseBlock + threadIdx.x;
  double s = 0.0;
  for (int i0 = 0; i0 < m; i0 += kPhaseBlock) {
    const int i = i0 + threadIdx.x;
    s_cb[threadIdx.x] = i < m ? lp.chat[lp.basis[i]] : 0.0;
    __syncthreads();
    const int cnt = min(kPhaseBlock, m - i0);
    if (j < ld) {
      const double* col = lp.Binv + (size_t)i0 * ld + j;
      for (int k = 0; k < cnt; ++k) {
        const double cb = s_cb[k];
        if (cb != 0.0) s = fma(cb, col[(size_t)k * ld], s);
      }
    }
    __syncthreads();
  }
  if (j < ld) {
    lp.W0[j] = s;
    lp.W1[j] = s;
  }
}

// z = sum_i chat_{basis[i]} x_B[i] over the rows with a nonzero cost, ascending i: the
// workgroup stages (cost, x_B) pairs in LDS, one thread sums them in order.
__global__ __launch_bounds__(kZBlock) void k_reprice_z(DevLP lp) {
  __shared__ double s_p[2 * kZBlock];
  const int m = lp.m, tid = threadIdx.x;
  double z = 0.0;
  for (int i0 = 0; i0 < m; i0 += kZBlock) {
    const int i = i0 + tid;
    s_p[2 * tid] = i < m ? lp.chat[lp.basis[i]] : 0.0;
    s_p[2 * tid + 1] = i < m ? lp.xB[i] : 0.0;
    __syncthreads();
    if (tid == 0) {
      const int cnt = min(kZBlock, m - i0);
      for (int k = 0; k < cnt; ++k) {
        const double cb = s_p[2 * k];
        if (cb != 0.0) z = fma(cb, s_p[2 * k + 1], z);
      }
    }
    __syncthreads();
  }
  if (tid == 0) lp.ctrl->z = z;
}

// Row r of the tableau over the candidate columns (nonbasic and not barred): t_j =
// B^-1[r,:] a_j, an ascending fma chain per structural column, B^-1[r, i] for the unit
// column n+i.  Each workgroup leaves the candidate with the largest |t_j| above eps_p
// (lowest j on equal magnitude) as the lexicographic minimum of (-|t_j|, j).
__global__ __launch_bounds__(kPhaseBlock) void k_tabrow(DevLP lp, int r, double* part_t, int32_t* part_j) {
  extern __shared__ double s_row[];
  __shared__ double red_d[kPhaseBlock / 64];
  __shared__ int red_j[kPhaseBlock / 64];
  const int m = lp.m, n = lp.n, ld = lp.ld, N = n + m;
  for (int k = threadIdx.x; k < ld; k += kPhaseBlock) s_row[k] = lp.Binv[(size_t)r * ld + k];
  __syncthreads();
  double key = __builtin_inf();
  int bj = INT_MAX;
  for (int j = blockIdx.x * kPhaseBlock + threadIdx.x; j < N; j += gridDim.x * kPhaseBlock) {
    if (lp.pos[j] != -1) continue;
    double t;
    if (j < n) {
      const double* a = lp.A + (size_t)j * ld;
      double s = 0.0;
      for (int k = 0; k < m; ++k) s = fma(a[k], s_row[k], s);
      t = s;
    } else {
      t = s_row[j - n];
    }
    const double at = fabs(t);
    if (at > lp.eps_p && lex_less(-at, j, key, bj)) {
      key = -at;
      bj = j;
    }
  }
  block_lexmin<kPhaseBlock>(key, bj, red_d, red_j);
  if (threadIdx.x == 0) {
    part_t[blockIdx.x] = key;
    part_j[blockIdx.x] = bj;
  }
}

// drive[0] = the column chosen for row r, or -1 (a redundant row).
__global__ __launch_bounds__(kPhaseBlock) void k_drive_pick(const double* part_t, const int32_t* part_j, int nparts,
                                                            int32_t* drive) {
  __shared__ double red_d[kPhaseBlock / 64];
  __shared__ int red_j[kPhaseBlock / 64];
  double key = __builtin_inf();
  int bj = INT_MAX;
  for (int k = threadIdx.x; k < nparts; k += kPhaseBlock) {
    if (lex_less(part_t[k], part_j[k], key, bj)) {
      key = part_t[k];
      bj = part_j[k];
    }
  }
  block_lexmin<kPhaseBlock>(key, bj, red_d, red_j);
  if (threadIdx.x == 0) drive[0] = bj == INT_MAX ? -1 : bj;
}

// Step 5 for the chosen column q: alpha_i = B^-1[i,:] a_q (ascending fma chain, one thread
// per row), or B^-1[i, q-n] for a unit column; into alpha0.
__global__ __launch_bounds__(kPhaseBlock) void k_drive_alpha(DevLP lp, const int32_t* drive) {
  const int q = drive[0];
  const int i = blockIdx.x * kPhaseBlock + threadIdx.x;
  if (q < 0 || i >= lp.m) return;
  const int m = lp.m, n = lp.n, ld = lp.ld;
  const double* row = lp.Binv + (size_t)i * ld;
  double s;
  if (q < n) {
    const double* a = lp.A + (size_t)q * ld;
    s = 0.0;
    for (int k = 0; k < m; ++k) s = fma(row[k], a[k], s);
  } else {
    s = row[q - n];
  }
  lp.alpha0[i] = s;
}

// rho = B^-1[r,:] / alpha_r (zero on the padding).
__global__ __launch_bounds__(kPhaseBlock) void k_drive_rho(DevLP lp, int r, const int32_t* drive) {
  const int j = blockIdx.x * kPhaseBlock + threadIdx.x;
  if (drive[0] < 0 || j >= lp.ld) return;
  lp.rho[j] = j < lp.m ? lp.Binv[(size_t)r * lp.ld + j] / lp.alpha0[r] : 0.0;
}

// Step 8 on B^-1 with the step 0: row r := rho, rows i != r: fma(-alpha_i, rho_j, .);
// x_B[r] := 0 and the other entries of x_B keep their values.
__global__ __launch_bounds__(kPhaseBlock) void k_drive_update(DevLP lp, int r, const int32_t* drive) {
  if (drive[0] < 0) return;
  const int ld = lp.ld;
  const size_t total = (size_t)lp.m * ld;
  const size_t stride = (size_t)gridDim.x * kPhaseBlock;
  for (size_t k = blockIdx.x * (size_t)kPhaseBlock + threadIdx.x; k < total; k += stride) {
    const int i = (int)(k / ld), j = (int)(k - (size_t)i * ld);
    const double rj = lp.rho[j];
    lp.Binv[k] = i == r ? rj : fma(-lp.alpha0[i], rj, lp.Binv[k]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) lp.xB[r] = 0.0;
}

// Basis bookkeeping of the step-0 pivot: the artificial variable leaves for good; its
// unit column of B^-1 joins the list D; the pivot is logged with kFlagDriveOut.
__global__ void k_drive_book(DevLP lp, int r, const int32_t* drive) {
  const int q = drive[0];
  if (q < 0 || threadIdx.x != 0) return;
  Ctrl* ctl = lp.ctrl;
  const int leave = lp.basis[r];
  const int64_t t = ctl->t;
  const int col = leave - lp.n;
  if (!lp.inD[col]) {
    lp.inD[col] = 1;
    lp.dlist[ctl->nD] = col;
    ctl->nD += 1;
  }
  lp.basis[r] = q;
  lp.pos[q] = r;
  lp.pos[leave] = kPosBarred;
  if (q < lp.n) ctl->nsb += 1;
  if (t < lp.log_cap) {
    lp.log_enter[t] = q;
    lp.log_row[t] = r;
    lp.log_leave[t] = leave;
    lp.log_flags[t] = kFlagDriveOut;
  }
  ctl->t = t + 1;
}

}  // namespace

int tabrow_grid(const DevLP& lp) { return std::max(1, std::min(1024, (lp.n + lp.m + kPhaseBlock - 1) / kPhaseBlock)); }

hipError_t launch_reprice(const DevLP& lp, hipStream_t s) {
  hipLaunchKernelGGL(k_reprice_w, dim3((lp.ld + kPhaseBlock - 1) / kPhaseBlock), dim3(kPhaseBlock), 0, s, lp);
  hipLaunchKernelGGL(k_reprice_z, dim3(1), dim3(kZBlock), 0, s, lp);
  return hipGetLastError();
}

hipError_t launch_drive_out(const DevLP& lp, int r, double* part_t, int32_t* part_j, int32_t* drive, hipStream_t s) {
  const int g = tabrow_grid(lp);
  hipLaunchKernelGGL(k_tabrow, dim3(g), dim3(kPhaseBlock), sizeof(double) * lp.ld, s, lp, r, part_t, part_j);
  hipLaunchKernelGGL(k_drive_pick, dim3(1), dim3(kPhaseBlock), 0, s, (const double*)part_t,
                     (const int32_t*)part_j, g, drive);
  hipLaunchKernelGGL(k_drive_alpha, dim3((lp.m + kPhaseBlock - 1) / kPhaseBlock), dim3(kPhaseBlock), 0, s, lp,
                     (const int32_t*)drive);
  hipLaunchKernelGGL(k_drive_rho, dim3((lp.ld + kPhaseBlock - 1) / kPhaseBlock), dim3(kPhaseBlock), 0, s, lp, r,
                     (const int32_t*)drive);
  const size_t total = (size_t)lp.m * lp.ld;
  const int ug = (int)std::min<size_t>(4096, (total + kPhaseBlock - 1) / kPhaseBlock);
  hipLaunchKernelGGL(k_drive_update, dim3(ug), dim3(kPhaseBlock), 0, s, lp, r, (const int32_t*)drive);
  hipLaunchKernelGGL(k_drive_book, dim3(1), dim3(64), 0, s, lp, r, (const int32_t*)drive);
  return hipGetLastError();
}

}  // namespace lpgpu
