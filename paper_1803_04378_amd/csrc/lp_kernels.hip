// Kernels of one dense revised simplex iteration for CDNA4 (gfx950, wave64).
//
// An iteration is ordered only by kernel boundaries (no grid-wide fences, which cost an
// L2 write-back per workgroup on this part):
//   k_price   Step 8 on the top row for the previous pivot (W += d_q rho, formed while
//             staging W in LDS), then Steps 3-4: reduced costs d_j = chat_j - W a_j of
//             every nonbasic column, one wavefront per column of A'; each workgroup
//             leaves its lexicographic (d, j) minima over all improving and over
//             non-tabu improving columns.
//   k_update  every workgroup reduces those partials to the same q (Step 4), then runs
//             the Section 3.1 update of B^-1 and x_B for the previous pivot fused with
//             Step 5 (FTRAN, alpha = B^-1 a_q) for q: one wavefront per row of B^-1
//             reads the row once, writes the updated row, dots it with a_q on the fly,
//             and forms that row's ratio (Step 6); each workgroup leaves its minimum
//             ratio and its rows within the tie bound.  k_update_c does the same on the
//             compact columns of B^-1 (rows of 1024 and more), k_update on whole rows.
//   k_finish  one workgroup: Step 6 ties and tabu list, then the scalar part of Step 8
//             (basis, entering mask, objective, pivot log).
// In the FP64 form k_price_fin, run by every iteration of a launch sequence but the
// first, is k_finish's work for the previous iteration (in every workgroup) followed by
// k_price's: K iterations take 2K + 1 launches.
//
// The B^-1 update of pivot t therefore runs in the same pass as the FTRAN of pivot
// t+1.  This is legal because pricing for t+1 needs only W_{t+1} = W_t + d_q rho_t,
// which needs only row r of the not yet updated B^-1; it removes one full read of
// B^-1 per iteration.  Every element still gets the same arithmetic as in Step 8.
//
// Reductions are deterministic: each dot product is a fixed per-lane fma chain
// followed by a fixed xor-butterfly, and every argmin is a lexicographic (value,
// index) minimum, which does not depend on the order partials arrive in.  No
// floating-point atomics are used.
#include "lp_device.h"
#include "lp_wave.h"

#include <limits.h>

#include <algorithm>

namespace lpgpu {

using namespace detail;

// ---------------------------------------------------------------------------------------
// Slack basis (Step 1): B = I, x_B = b, W = 0, z = 0; chat = sense * c.
__global__ void k_init(DevLP lp, const double* __restrict__ b, const double* __restrict__ c, double sense) {
  const int m = lp.m, n = lp.n, ld = lp.ld, N = n + m;
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  // (out-of-core panel mode: B^-1 lives in host memory and is set up by the host)
  const size_t total = lp.Binv ? (size_t)m * ld : 0;
  for (size_t k = tid; k < total; k += stride) {
    const size_t i = k / ld, j = k - i * ld;
    lp.Binv[k] = (i == j) ? 1.0 : 0.0;
  }
  // compact columns: D is empty, every column of Bc zero
  const size_t ctotal = lp.cmode ? (size_t)m * ld : 0;
  for (size_t k = tid; k < ctotal; k += stride) lp.Bc[k] = 0.0;
  for (size_t k = tid; k < (size_t)ld; k += stride) {
    lp.W0[k] = 0.0;
    lp.W1[k] = 0.0;
    lp.rho[k] = 0.0;
  }
  for (size_t i = tid; i < (size_t)m; i += stride) {
    lp.xB[i] = b[i];
    lp.inD[i] = 0;
    lp.basis[i] = n + (int)i;
    lp.alpha0[i] = 0.0;
    lp.alpha1[i] = 0.0;
  }
  double* chat = const_cast<double*>(lp.chat);
  for (size_t v = tid; v < (size_t)N; v += stride) {
    chat[v] = v < (size_t)n ? sense * c[v] : 0.0;
    lp.pos[v] = v < (size_t)n ? -1 : (int)(v - n);
    lp.tabu_until[v] = -1;
    lp.gen[v] = 0;
    lp.excl[v] = -1;
  }
  if (tid == 0) {
    Ctrl* ctl = lp.ctrl;
    *ctl = Ctrl{};
    ctl->status = kStatusRunning;
    ctl->q = -1;
    ctl->r = -1;
    ctl->ray = -1;
    ctl->verdict = -1;
    ctl->gen_q = -1;
    ctl->dapp = -1;
    ctl->ind_pend = -1;
  }
}

// ---------------------------------------------------------------------------------------
// Inputs and result of the ratio-test finish (finish_step, below).
struct FinishIn {
  int verdict, q, cur, flags0, nD0, nsb0, nL;
  int64_t t;
  double dq, z0;
};
struct FinishOut {
  int pivot;  // 1: a pivot on row r was committed; 0: the solve stopped or (mixed) no pivot
  int r, leave;
  int kept;  // 0: the leaving slack's column joined D (at index nD0)
  double ar;
};

template <int B, bool FUSED>
__device__ FinishOut finish_step(const DevLP& lp, const FinishIn& in, double pth, double pt1, double pt2, double pal,
                                 int plow, int pbv);

// Steps 3-4, preceded by Step 8 on the top row of the tableau for the pending pivot:
// every workgroup forms W_new = W + d_q rho, rho = B^-1[r,:] / alpha_r, while staging it
// into LDS (B^-1 still holds the pre-pivot rows, the row update runs in k_update);
// workgroup 0 also stores rho and W_new for the rest of the iteration.  (The mixed form
// does not launch this kernel: k_price32 screens, and runs the FP64 pass when needed.)
//
// FUSED (k_price_fin): the pending pivot is the one this kernel finishes first from
// k_update's partials (finish_step, in every workgroup).  Its bookkeeping may or may not
// be visible to a workgroup yet, so the entering variable counts as basic and the leaving
// one as nonbasic (and tabu) whatever pos and tabu_until read.
// NT: A' is read with non-temporal loads (it does not fit the 256 MB last-level cache, so
// lines kept would be evicted before the next pass reads them); else with ordinary loads,
// which let A' stay in that cache from one pricing pass to the next.
template <bool FUSED, bool NT>
__device__ __forceinline__ void price_pass(const DevLP& lp, double2* s_w2) {
  __shared__ double red_d[2 * (kPriceBlock / 64)];
  __shared__ int red_j[2 * (kPriceBlock / 64)];
  const int m = lp.m, n = lp.n, ld2 = lp.ld / 2;
  constexpr int waves = kPriceBlock / 64;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gw = blockIdx.x * waves + wave;
  const int nw = gridDim.x * waves;

  // Requested together, before anything waits on memory: the control block (in the fused
  // kernel also the first update partial of every thread), the state of this wave's
  // columns (lane c holds column gw + c*nw) and the first batch of its first column of A'
  // (read even when the solve has stopped; then unused).
  const Ctrl* ctl = lp.ctrl;
  const int status = ctl->status;
  const int wc = ctl->wcur;
  int64_t t;
  int r;
  double ar, dq;
  FinishIn fin;
  double pth = 0.0, pt1 = 0.0, pt2 = 0.0, pal = 0.0;
  int plow = 0, pbv = 0;
  if (FUSED) {
    fin.verdict = ctl->verdict;
    fin.q = ctl->q;
    fin.cur = ctl->snap_cur;
    fin.t = ctl->snap_t;
    fin.flags0 = ctl->flags;
    fin.dq = ctl->dq;
    fin.z0 = ctl->snap_z;
    fin.nD0 = ctl->snap_nD;
    fin.nsb0 = ctl->snap_nsb;
    fin.nL = ctl->snap_nL;
    const int pk = min((int)threadIdx.x, lp.update_grid - 1);
    pth = lp.part_th[pk];
    pt1 = lp.part_t1[pk];
    pt2 = lp.part_t2[pk];
    pal = lp.part_al[pk];
    plow = lp.part_low[pk];
    pbv = lp.part_bv[pk];
    t = fin.t + 1;
    dq = fin.dq;
    r = -1;
    ar = 0.0;
  } else {
    t = ctl->t;
    r = ctl->r;
    ar = ctl->ar;
    dq = ctl->pdq;
  }
  // compact columns: the length of D after the pending pivot, and the index it appended
  int nDn = 0, a_app = -1, j_app = -1;
  if (!FUSED && lp.cmode) {
    nDn = ctl->nD;
    a_app = ctl->dapp;
  }
  const int jl = gw + lane * nw;
  int c_pos = 0, c_tabu = 0;
  double c_chat = 0.0;
  if (jl < n) {
    c_pos = lp.pos[jl];
    c_tabu = lp.tabu_until[jl];
    c_chat = lp.chat[jl];
  }
  double2 v[kBatch];
  const bool pre = gw < n;
  if (pre) {
    if (NT) load_batch_nt(reinterpret_cast<const double2*>(lp.A + (size_t)gw * lp.ld), lane, ld2, v);
    else load_batch(reinterpret_cast<const double2*>(lp.A + (size_t)gw * lp.ld), lane, ld2, v);
  }
  if (FUSED) asm volatile("" ::: "memory");  // compiler-only: all of the above is requested first
  if (status != kStatusRunning) return;

  // The pivot just finished (fused): its entering and leaving variables, and the leaving
  // one's view of pos and tabu_until after the pivot.
  int pq = -1, pl = -1, pl_pos = 0, pl_tabu = 0;
  if (FUSED) {
    const FinishOut fo = finish_step<kPriceBlock, true>(lp, fin, pth, pt1, pt2, pal, plow, pbv);
    if (!fo.pivot) return;
    r = fo.r;
    ar = fo.ar;
    pq = fin.q;
    pl = fo.leave;
    pl_pos = (lp.art && pl >= n && lp.art[pl - n]) ? kPosBarred : -1;
    pl_tabu = lp.tenure > 0 ? (int)(fin.t + lp.tenure) : lp.tabu_until[pl];
    // (dlist[nD0] is written by workgroup 0 in this launch: the appended column is pl - n)
    nDn = fin.nD0 + (fo.kept ? 0 : 1);
    a_app = fo.kept ? -1 : fin.nD0;
    j_app = pl - n;
  }

  if (r >= 0 && lp.cmode) {
    // Compact columns: rho = B^-1[r,:] / alpha_r is zero outside D, and row r of Bc holds
    // it on D (at the appended index the unit column's 1, not stored yet).  W is staged as
    // it is, then W + d_q rho is formed at the columns of D: the same values as the dense
    // formation, which leaves every other entry unchanged.  Workgroup 0 stores rho_c and
    // W_new.
    const double2* Wold = reinterpret_cast<const double2*>(wc ? lp.W1 : lp.W0);
    double2* Wnew = reinterpret_cast<double2*>(wc ? lp.W0 : lp.W1);
    const double* crow = lp.Bc + (size_t)r * lp.ld;
    const bool writer = blockIdx.x == 0;
    const int a0 = threadIdx.x, a1 = threadIdx.x + kPriceBlock;
    double b0 = 0.0, b1 = 0.0;
    int j0 = 0, j1 = 0;
    if (a0 < nDn) {
      b0 = crow[a0];
      j0 = lp.dlist[a0];
    }
    if (a1 < nDn) {
      b1 = crow[a1];
      j1 = lp.dlist[a1];
    }
    for (int k = threadIdx.x; k < ld2; k += kPriceBlock) s_w2[k] = Wold[k];
    __syncthreads();
    double* s_wd = reinterpret_cast<double*>(s_w2);
    auto apply = [&](int a, double b, int j) {
      if (a == a_app) {
        b = 1.0;
        if (FUSED) j = j_app;
      }
      const double rr = b / ar;
      s_wd[j] = fma(dq, rr, s_wd[j]);
      if (writer) lp.rho_c[a] = rr;
    };
    if (a0 < nDn) apply(a0, b0, j0);
    if (a1 < nDn) apply(a1, b1, j1);
    for (int a = a1 + kPriceBlock; a < nDn; a += kPriceBlock) apply(a, crow[a], lp.dlist[a]);
    __syncthreads();
    if (writer)
      for (int k = threadIdx.x; k < ld2; k += kPriceBlock) Wnew[k] = s_w2[k];
  } else if (r >= 0) {
    const double2* Wold = reinterpret_cast<const double2*>(wc ? lp.W1 : lp.W0);
    // row r of B^-1: in the out-of-core panel mode a device copy fetched after the ratio test
    const double2* rowr = reinterpret_cast<const double2*>(lp.rowsrc ? lp.rowsrc : lp.Binv + (size_t)r * lp.ld);
    double2* Wnew = reinterpret_cast<double2*>(wc ? lp.W0 : lp.W1);
    double2* rho2 = reinterpret_cast<double2*>(lp.rho);
    const bool writer = blockIdx.x == 0;
    int nz2 = 0;
    for (int k = threadIdx.x; k < ld2; k += kPriceBlock) {
      const double2 b = rowr[k];
      const double2 w = Wold[k];
      const double2 rr = make_double2(b.x / ar, b.y / ar);
      const double2 wn = make_double2(fma(dq, rr.x, w.x), fma(dq, rr.y, w.y));
      s_w2[k] = wn;
      if (writer) {
        rho2[k] = rr;
        Wnew[k] = wn;
        nz2 += (rr.x != 0.0 || rr.y != 0.0) ? 1 : 0;
      }
    }
    if (writer) {
      nz2 = block_sum_int<kPriceBlock>(nz2, red_j);
      if (threadIdx.x == 0) lp.ctrl->rho_nz2 = nz2;
    }
  } else {
    // the top row to price with (as pricing_w)
    const double2* W2 = reinterpret_cast<const double2*>((wc != 0) != (r >= 0) ? lp.W1 : lp.W0);
    for (int k = threadIdx.x; k < ld2; k += kPriceBlock) s_w2[k] = W2[k];
  }
  __syncthreads();
  const double* s_w = reinterpret_cast<const double*>(s_w2);

  const double neg_eps = -lp.eps_d;
  double da = __builtin_inf(), df = __builtin_inf();
  int ja = INT_MAX, jf = INT_MAX;
  int c = 0;
  for (int j = gw; j < n; j += nw, ++c) {
    int pos, tabu;
    double ch;
    if (c < 64) {
      pos = __shfl(c_pos, c);
      tabu = __shfl(c_tabu, c);
      ch = __shfl(c_chat, c);
    } else {
      pos = lp.pos[j];
      tabu = lp.tabu_until[j];
      ch = lp.chat[j];
    }
    if (FUSED) {
      if (j == pq) pos = r;
      if (j == pl) {
        pos = pl_pos;
        tabu = pl_tabu;
      }
    }
    const bool first = c == 0;
    if (pos >= 0) continue;
    const double s = wave_dot<NT>(reinterpret_cast<const double2*>(lp.A + (size_t)j * lp.ld), s_w2, ld2,
                                        lane, v, first && pre);
    const double d = ch - s;
    if (d < neg_eps) {
      if (lex_less(d, j, da, ja)) {
        da = d;
        ja = j;
      }
      if (tabu < t && lex_less(d, j, df, jf)) {
        df = d;
        jf = j;
      }
    }
  }
  for (int i = blockIdx.x * kPriceBlock + threadIdx.x; i < m; i += gridDim.x * kPriceBlock) {
    const int vv = n + i;
    int pos = lp.pos[vv], tabu = lp.tabu_until[vv];
    if (FUSED) {
      if (vv == pq) pos = r;
      if (vv == pl) {
        pos = pl_pos;
        tabu = pl_tabu;
      }
    }
    if (pos >= 0) continue;
    const double d = lp.chat[vv] - s_w[i];  // a_{n+i} = e_i
    if (d < neg_eps) {
      if (lex_less(d, vv, da, ja)) {
        da = d;
        ja = vv;
      }
      if (tabu < t && lex_less(d, vv, df, jf)) {
        df = d;
        jf = vv;
      }
    }
  }
  // Workgroup partials: both minima through one LDS exchange.
  wave_lexmin(da, ja);
  wave_lexmin(df, jf);
  if (lane == 0) {
    red_d[wave] = da;
    red_j[wave] = ja;
    red_d[waves + wave] = df;
    red_j[waves + wave] = jf;
  }
  __syncthreads();
  if (wave == 0) {
    da = lane < waves ? red_d[lane] : __builtin_inf();
    ja = lane < waves ? red_j[lane] : INT_MAX;
    df = lane < waves ? red_d[waves + lane] : __builtin_inf();
    jf = lane < waves ? red_j[waves + lane] : INT_MAX;
    wave_lexmin(da, ja);
    wave_lexmin(df, jf);
    if (lane == 0) {
      lp.part_d[2 * blockIdx.x] = da;
      lp.part_j[2 * blockIdx.x] = ja;
      lp.part_d[2 * blockIdx.x + 1] = df;
      lp.part_j[2 * blockIdx.x + 1] = jf;
    }
  }
}

template <bool NT>
__global__ __launch_bounds__(kPriceBlock) void k_price(DevLP lp) {
  extern __shared__ double2 s_w2[];
  price_pass<false, NT>(lp, s_w2);
}

// The ratio-test finish of the pending iteration (k_finish's work, in every workgroup)
// fused with the next pricing pass: one launch instead of two, and the finish's loads
// overlap the first batch of A'.
// Held to k_price's register budget (six waves per SIMD), so that the grid sized for
// k_price stays resident in one round.
template <bool NT>
__global__ __launch_bounds__(kPriceBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_price_fin(DevLP lp) {
  extern __shared__ double2 s_w2[];
  price_pass<true, NT>(lp, s_w2);
}

// ---------------------------------------------------------------------------------------
// Section 3.1 update of the pending pivot (rows of B^-1 and x_B) fused with Step 5 for
// the newly priced q and with the per-row part of Step 6.  Every workgroup first reduces
// the pricing partials itself (a lexicographic minimum, so all of them agree on q).
//
// The kernel is short on data and long on dependent memory accesses, so it is laid out
// as two rounds of requests: first everything that depends only on earlier kernels (the
// control block, the pricing partials or the shortlist, rho, the head of list D, the
// state of this wavefront's first row), then what depends on q (the column a_q, the row
// entries of sparse mode).  rho and a_q are staged whole in LDS, so the sparse mode's
// per-column lookups and the unit term of a row's basic slack are LDS reads.

// A vector of up to kUpdRegs * kUpdateBlock double2 loaded by one workgroup into
// registers, up to kUpdRegs per thread, with clamped indices inside a chunk (no lane-level
// branch for a load to wait behind); hold_store copies any longer tail directly.
// Held as native vectors: copies of the double2 struct go through a stack temporary.
#ifndef LPGPU_UPD_REGS
#define LPGPU_UPD_REGS 5
#endif
constexpr int kUpdRegs = LPGPU_UPD_REGS;
struct Hold5 {
  v2d h[kUpdRegs];
};
// Load batch of the dense row update: 4 double2 per lane (the 8 of the streaming kernels
// would not leave room for the staged vectors within 128 VGPRs).
constexpr int kUpdBatch = 4;
// Chunks wholly beyond n2 are skipped (a condition uniform over the workgroup, so no
// lane-level branch); h.h[u] is then undefined and hold_store does not read it.
template <int B>
__device__ __forceinline__ void hold_load(Hold5& h, const double2* __restrict__ src2, int tid, int n2) {
  const v2d* src = reinterpret_cast<const v2d*>(src2);
  h.h[0] = src[min(tid, n2 - 1)];
#pragma unroll
  for (int u = 1; u < kUpdRegs; ++u)
    if (u * B < n2) h.h[u] = src[min(tid + u * B, n2 - 1)];
}
// Stores what hold_load read into dst (LDS), then copies any part beyond kUpdRegs * kUpdateBlock.
template <int B>
__device__ __forceinline__ void hold_store(const Hold5& h, double2* dst2, const double2* __restrict__ src2, int tid,
                                           int n2) {
  v2d* dst = reinterpret_cast<v2d*>(dst2);
  const v2d* src = reinterpret_cast<const v2d*>(src2);
#pragma unroll
  for (int u = 0; u < kUpdRegs; ++u)
    if (tid + u * B < n2) dst[tid + u * B] = h.h[u];
  for (int k = tid + kUpdRegs * B; k < n2; k += B) dst[k] = src[k];
}
// Entries of list D per lane gathered from a row in one round (nD <= 512); the rest, if
// any, follow in a loop.
constexpr int kGather = 8;

template <int B>
__global__ __launch_bounds__(B) void k_update(DevLP lp) {
  constexpr int waves = B / 64;
  extern __shared__ double2 smem2[];
  __shared__ double red_d[2 * waves];
  __shared__ int red_j[2 * waves];
  __shared__ double s_rt[waves * kMaxRowsPerWave];
  __shared__ double s_tau[waves * kMaxRowsPerWave];
  __shared__ int s_row[waves * kMaxRowsPerWave];
  __shared__ double s_al[waves * kMaxRowsPerWave];
  __shared__ int s_bv[waves * kMaxRowsPerWave];
  __shared__ int s_nf;  // some row of this workgroup has a non-finite alpha
  const int m = lp.m, n = lp.n, ld = lp.ld, ld2 = ld / 2;
  // Rows lo..hi-1 of B^-1, row i at Binv + (i - lo) ld: all of them, or one panel of the
  // out-of-core mode (a launch per panel; the first one also does the iteration's
  // bookkeeping in the control block).
  const int lo = lp.row_lo, hi = lp.row_hi;
  const bool first_panel = lo == 0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_nf = 0;  // read after the barriers below
  const int gw = blockIdx.x * waves + wave;
  const int nw = gridDim.x * waves;
  double2* s_rho = smem2;
  double2* s_a = smem2 + ld2;
  int* s_dl = reinterpret_cast<int*>(smem2 + 2 * ld2);
  // Sparse mode reads at most ld/8 entries of D (<= m, the list's capacity); below
  // kSparseMinLd the update is always dense.
  const bool can_sparse = ld >= kSparseMinLd;
  const int dcap = can_sparse ? ld / 8 : 0;

  // ---- first round: requests that depend only on the previous kernels ----
  const Ctrl* ctl = lp.ctrl;
  const int status = ctl->status;
  const int r = ctl->r;
  const int nD = ctl->nD;
  const int cur = ctl->cur;
  const int64_t t = ctl->t;
  const int64_t max_iter = ctl->max_iter;
  const double theta = ctl->theta;
  const int fb = ctl->fb;
  // basis[r] of a pivot k_price_fin finished is written below; until then it reads as q_pend
  const int bpend = ctl->bpend, q_pend = ctl->q_pend;
  // Indices are clamped into range rather than guarded, so that no load waits behind a
  // branch; the values of clamped lanes are discarded below.
  const int pk = min(tid, lp.price_grid - 1);
  double pd0 = lp.part_d[2 * pk], pd1 = lp.part_d[2 * pk + 1];
  int pj0 = lp.part_j[2 * pk], pj1 = lp.part_j[2 * pk + 1];
  const double2* rho2 = reinterpret_cast<const double2*>(lp.rho);
  Hold5 hold;
  hold_load<B>(hold, rho2, tid, ld2);  // unused if no pivot is pending
  int dl0 = 0, dl1 = 0;
  if (can_sparse) {
    dl0 = lp.dlist[min(tid, dcap - 1)];
    dl1 = lp.dlist[min(tid + B, dcap - 1)];
  }
  const int i0 = lo + gw;  // this wavefront's first row
  const int g0 = min(i0, hi - 1);
  double x0 = lp.xB[g0], al00 = lp.alpha0[g0], al10 = lp.alpha1[g0];
  int bv0 = lp.basis[g0];
  if (bpend && g0 == r) bv0 = q_pend;
  double2 v[kUpdBatch];
  const bool pre_now = !can_sparse && i0 < hi;  // dense for certain: first batch of the row now
  if (pre_now) load_batch(reinterpret_cast<const double2*>(lp.Binv + (size_t)gw * ld), lane, ld2, v);
  double sd = __builtin_inf();
  int sj = INT_MAX;
  if (lp.mixed) {
    const int w = min(lane, lp.sl_k - 1);
    sd = lp.sl_d[w];
    sj = lp.sl_j[w];
  }
  // Compiler-only barrier (no instruction): every request above is issued before any of
  // the code below waits on one.
  asm volatile("" ::: "memory");
  if (tid >= lp.price_grid) {
    pd0 = pd1 = __builtin_inf();
    pj0 = pj1 = INT_MAX;
  }

  hold_store<B>(hold, s_rho, rho2, tid, ld2);
  if (tid < dcap) s_dl[tid] = dl0;
  if (tid + B < dcap) s_dl[tid + B] = dl1;

  // Step 4 decision: in the mixed form from the re-priced shortlist (none improving: the
  // fallback verdict below), else, and in the mixed form's FP64 pass, from the pricing
  // partials.
  double da = __builtin_inf(), df = __builtin_inf();
  int ja = INT_MAX, jf = INT_MAX;
  bool from_shortlist = false;
  const bool use_parts = !lp.mixed || fb;
  if (lp.mixed && !fb) {
    // the best improving column of the re-priced shortlist: lane w reads entry w, a
  // wavefront minimum combines them (its columns are all non-tabu)
    if (!(lane < lp.sl_k && sj != INT_MAX && sd < -lp.eps_d)) {
      sd = __builtin_inf();
      sj = INT_MAX;
    }
    wave_lexmin(sd, sj);
    df = sd;
    jf = sj;
    from_shortlist = jf != INT_MAX;
    da = df;
    ja = jf;
  }
  if (use_parts) {
    da = pd0;
    ja = pj0;
    df = pd1;
    jf = pj1;
    for (int k = tid + B; k < lp.price_grid; k += B) {
      const double d0 = lp.part_d[2 * k], d1 = lp.part_d[2 * k + 1];
      const int j0 = lp.part_j[2 * k], j1 = lp.part_j[2 * k + 1];
      if (lex_less(d0, j0, da, ja)) {
        da = d0;
        ja = j0;
      }
      if (lex_less(d1, j1, df, jf)) {
        df = d1;
        jf = j1;
      }
    }
    wave_lexmin(da, ja);
    wave_lexmin(df, jf);
    if (lane == 0) {
      red_d[wave] = da;
      red_j[wave] = ja;
      red_d[waves + wave] = df;
      red_j[waves + wave] = jf;
    }
    __syncthreads();
    da = lane < waves ? red_d[lane] : __builtin_inf();
    ja = lane < waves ? red_j[lane] : INT_MAX;
    df = lane < waves ? red_d[waves + lane] : __builtin_inf();
    jf = lane < waves ? red_j[waves + lane] : INT_MAX;
    wave_lexmin(da, ja);  // every wave reduces the same values: no second exchange needed
    wave_lexmin(df, jf);
  }
  __syncthreads();  // rho and D are in LDS
  if (status != kStatusRunning) return;
  // (the first 2B entries of D are staged above: ld/8 exceeds 2B only for 512-thread
  // workgroups above ld = 8192, where a longer list takes the dense pass)
  const bool sparse = sparse_columns(nD, ld) && nD <= 2 * B;
  int verdict = kStatusRunning, q = -1, flags = 0;
  double dq = 0.0;
  if (!use_parts && !from_shortlist) {
    verdict = kVerdictFallback;
  } else if (ja == INT_MAX) {
    verdict = kStatusOptimal;
  } else if (t >= max_iter) {
    verdict = kStatusIterLimit;
  } else if (jf != INT_MAX) {
    q = jf;
    dq = df;
  } else {
    q = ja;
    dq = da;
    flags = kFlagAspiration;
  }
  if (blockIdx.x == 0 && tid == 0 && first_panel) {
    // Only fields no k_update workgroup reads: the status itself changes in k_finish.
    Ctrl* cw = lp.ctrl;
    // (bpend outlives its pivot: after a stop, a reinversion or the phase switch r is -1)
    if (bpend && r >= 0) lp.basis[r] = q_pend;
    if (cw->gen_q >= 0) {
      lp.gen[cw->gen_q] = cw->gen_val;
      cw->gen_q = -1;
    }
    if (cw->ind_pend >= 0) {  // (no row of this launch has that slack basic)
      lp.inD[cw->ind_pend] = 1;
      cw->ind_pend = -1;
    }
    cw->snap_t = t;
    cw->snap_z = cw->z;
    cw->snap_nD = nD;
    cw->snap_nsb = cw->nsb;
    cw->snap_nL = cw->nL;
    cw->snap_cur = cur;
    if (lp.mixed && !fb) cw->price32_launches += 1;
    if (use_parts) {
      cw->price_cols += n - cw->nsb;
      cw->price_launches += 1;
      if (lp.mixed) cw->full_prices += 1;
    }
    if (r >= 0) cw->wcur ^= 1;  // pricing stored W_new: it is the current top row now
    cw->verdict = verdict;
    cw->q = q;
    cw->dq = dq;
    cw->flags = flags;
    if (flags & kFlagAspiration) cw->n_aspiration += 1;
    if (r >= 0) {
      cw->update_launches += 1;
      cw->update_rows_written += m;
    } else if (q >= 0) {
      cw->update_launches += 1;
    }
    if (!sparse && (r >= 0 || q >= 0)) {
      // read all of B^-1; write the pairs with a nonzero rho entry in every row but r,
      // and all of row r
      cw->update_bytes += 8 * (int64_t)m * m;
      if (r >= 0) cw->update_bytes += 16 * ((int64_t)(m - 1) * cw->rho_nz2 + ld / 2);
    }
  }
  if (r < 0 && q < 0) return;

  // ---- second round: a_q, and this wave's first row where it depends on D ----
  const double* __restrict__ al_p = cur ? lp.alpha1 : lp.alpha0;  // pending pivot's alpha
  double* __restrict__ al_n = cur ? lp.alpha0 : lp.alpha1;        // FTRAN result for q
  const double eps_p = lp.eps_p, eps_z = lp.eps_z;
  const bool q_col = q >= 0 && q < n;
  const double2* aq2 = reinterpret_cast<const double2*>(lp.A + (size_t)(q_col ? q : 0) * ld);
  if (q_col) hold_load<B>(hold, aq2, tid, ld2);
  const double* s_rhod = reinterpret_cast<const double*>(s_rho);
  const double* s_ad = reinterpret_cast<const double*>(s_a);
  // whether the first row's basic variable is a slack outside D (its B^-1 column is a
  // unit vector): the sparse FTRAN adds its unit term, and k_finish needs it for the
  // leaving variable
  int in0 = 1;
  if (i0 < hi && bv0 >= n) in0 = lp.inD[bv0 - n];
  int c = 0;
  if (sparse) {
    double g[kGather];
    if (i0 < hi) {
      const double* row = lp.Binv + (size_t)gw * ld;
#pragma unroll
      for (int u = 0; u < kGather; ++u) {
        const int a = lane + 64 * u;
        if (a < nD) g[u] = row[s_dl[a]];
      }
    }
    if (q_col) {
      hold_store<B>(hold, s_a, aq2, tid, ld2);
    } else if (q >= 0) {
      const int e = q - n;
      for (int k = tid; k < ld2; k += B) s_a[k] = make_double2(2 * k == e ? 1.0 : 0.0, 2 * k + 1 == e ? 1.0 : 0.0);
    }
    if (blockIdx.x == 0 && first_panel) {
      // bytes: D entries read in every row but r, the changed ones written in every
      // row, and one unit lookup (basis, membership, a_q entry) per row
      int nz = 0;
      if (r >= 0)
        for (int a = tid; a < nD; a += B) nz += s_rhod[s_dl[a]] != 0.0 ? 1 : 0;
      nz = block_sum_int<B>(nz, red_j);
      if (tid == 0) lp.ctrl->update_bytes += 8 * ((int64_t)(m - 1) * nD + (int64_t)m * nz) + 16 * (int64_t)m;
    }
    __syncthreads();  // a_q is in LDS
    for (int i = i0; i < hi; i += nw, ++c) {
      double* row = lp.Binv + (size_t)(i - lo) * ld;
      double x, alp;
      int bv, in;
      if (c == 0) {
        x = x0;
        alp = cur ? al10 : al00;
        bv = bv0;
        in = in0;
      } else {
        x = lp.xB[i];
        alp = al_p[i];
        bv = (bpend && i == r) ? q_pend : lp.basis[i];
        in = bv >= n ? lp.inD[bv - n] : 1;
#pragma unroll
        for (int u = 0; u < kGather; ++u) {
          const int a = lane + 64 * u;
          if (a < nD) g[u] = row[s_dl[a]];
        }
      }
      const bool isr = i == r;
      const double na = (r >= 0 && !isr) ? -alp : 0.0;
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < kGather; ++u) {
        const int a = lane + 64 * u;
        if (a < nD) {
          const int j = s_dl[a];
          double val = g[u];
          if (r >= 0) {
            const double rr = s_rhod[j];
            val = isr ? rr : fma(na, rr, val);  // row r := rho (zero wherever rho is zero)
            if (rr != 0.0) row[j] = val;
          }
          if (q >= 0) acc = fma(val, s_ad[j], acc);
        }
      }
      for (int a = lane + 64 * kGather; a < nD; a += 64) {
        const int j = s_dl[a];
        double val = row[j];
        if (r >= 0) {
          const double rr = s_rhod[j];
          val = isr ? rr : fma(na, rr, val);
          if (rr != 0.0) row[j] = val;
        }
        if (q >= 0) acc = fma(val, s_ad[j], acc);
      }
      if (r >= 0) {
        x = isr ? theta : fma(na, theta, x);
        if (fabs(x) < eps_z) x = 0.0;
        if (lane == 0) lp.xB[i] = x;
      }
      if (q >= 0) {
        acc = wave_sum(acc);
        // the unit column of this row's basic slack, when it is not in D
        if (bv >= n && !in) acc += s_ad[bv - n];
        double rt = __builtin_inf(), tau = __builtin_inf();
        if (acc > eps_p) {
          const double xp = fmax(x, 0.0);
          rt = xp / acc;
          tau = (xp - lp.eps_t) / acc;
          tau -= 1e-12 * (fabs(tau) + 1.0);
        }
        if (lane == 0) {
          al_n[i] = acc;
          s_rt[wave * kMaxRowsPerWave + c] = rt;
          s_tau[wave * kMaxRowsPerWave + c] = tau;
          s_row[wave * kMaxRowsPerWave + c] = acc > eps_p ? i : INT_MAX;  // INT_MAX: not a candidate
          if (!isfinite(acc)) s_nf = 1;
          s_al[wave * kMaxRowsPerWave + c] = acc;
          s_bv[wave * kMaxRowsPerWave + c] = 2 * bv + ((bv < n || in) ? 1 : 0);
        }
      }
    }
  } else {
    // dense mode with rows long enough for sparse mode: the first batch of the row now
    const bool pre_late = can_sparse && i0 < hi;
    if (pre_late) load_batch(reinterpret_cast<const double2*>(lp.Binv + (size_t)gw * ld), lane, ld2, v);
    if (q_col) {
      hold_store<B>(hold, s_a, aq2, tid, ld2);
    } else if (q >= 0) {
      const int e = q - n;
      for (int k = tid; k < ld2; k += B) s_a[k] = make_double2(2 * k == e ? 1.0 : 0.0, 2 * k + 1 == e ? 1.0 : 0.0);
    }
    __syncthreads();  // a_q is in LDS
    const bool pre = pre_now || pre_late;
    for (int i = i0; i < hi; i += nw, ++c) {
      double2* row = reinterpret_cast<double2*>(lp.Binv + (size_t)(i - lo) * ld);
      const bool first = c == 0 && pre;
      double acc;
      double x = c == 0 ? x0 : lp.xB[i];
      int bv = bv0, in = in0;
      if (c > 0 && q >= 0) {
        bv = (bpend && i == r) ? q_pend : lp.basis[i];
        in = bv >= n ? lp.inD[bv - n] : 1;
      }
      if (r < 0) {
        acc = wave_dot<false>(row, s_a, ld2, lane, v, first);
      } else {
        if (i == r) {
          acc = q >= 0 ? wave_store_dot<true>(row, s_rho, s_a, ld2, lane)
                       : wave_store_dot<false>(row, s_rho, s_a, ld2, lane);
          x = theta;
        } else {
          const double na = -(c == 0 ? (cur ? al10 : al00) : al_p[i]);
          acc = q >= 0 ? wave_update_dot<true>(row, s_rho, s_a, na, ld2, lane, v, first)
                       : wave_update_dot<false>(row, s_rho, s_a, na, ld2, lane, v, first);
          x = fma(na, theta, x);
        }
        if (fabs(x) < eps_z) x = 0.0;
        if (lane == 0) lp.xB[i] = x;
      }
      if (q >= 0) {
        // ratio_i, and tau_i: the smallest step at which row i would count as tied
        // (fma(-alpha_i, step, max(x_i, 0)) <= eps_t), lowered by a margin so that the
        // filter in k_finish never misses a tied row.
        double rt = __builtin_inf(), tau = __builtin_inf();
        if (acc > eps_p) {
          const double xp = fmax(x, 0.0);
          rt = xp / acc;
          tau = (xp - lp.eps_t) / acc;
          tau -= 1e-12 * (fabs(tau) + 1.0);
        }
        if (lane == 0) {
          al_n[i] = acc;
          s_rt[wave * kMaxRowsPerWave + c] = rt;
          s_tau[wave * kMaxRowsPerWave + c] = tau;
          s_row[wave * kMaxRowsPerWave + c] = acc > eps_p ? i : INT_MAX;  // INT_MAX: not a candidate
          if (!isfinite(acc)) s_nf = 1;
          s_al[wave * kMaxRowsPerWave + c] = acc;
          s_bv[wave * kMaxRowsPerWave + c] = 2 * bv + ((bv < n || in) ? 1 : 0);
        }
      }
    }
  }
  if (q < 0) return;
  // Workgroup partial of Step 6: (min ratio, lowest row attaining it) and the two
  // smallest tau of the workgroup's rows.
  for (int k = c; k < kMaxRowsPerWave; ++k)
    if (lane == 0) {
      s_rt[wave * kMaxRowsPerWave + k] = __builtin_inf();
      s_tau[wave * kMaxRowsPerWave + k] = __builtin_inf();
      s_row[wave * kMaxRowsPerWave + k] = INT_MAX;
    }
  __syncthreads();
  if (wave == 0) {
    constexpr int slots = waves * kMaxRowsPerWave;
    double th = __builtin_inf(), t1 = __builtin_inf(), t2 = __builtin_inf();
    int low = INT_MAX, slot = 0;
    for (int k = lane; k < slots; k += 64) {
      if (lex_less(s_rt[k], s_row[k], th, low)) {
        th = s_rt[k];
        low = s_row[k];
        slot = k;
      }
      const double tk = s_tau[k];
      if (tk < t1) {
        t2 = t1;
        t1 = tk;
      } else if (tk < t2) {
        t2 = tk;
      }
    }
    wave_lexmin_payload(th, low, slot);
    wave_two_smallest(t1, t2);
    if (lane == 0) {
      // a non-finite alpha is published as (-inf, -1), which no ratio (>= 0) undercuts
      lp.part_th[blockIdx.x] = s_nf ? -__builtin_inf() : th;
      lp.part_low[blockIdx.x] = s_nf ? -1 : low;
      lp.part_t1[blockIdx.x] = t1;
      lp.part_t2[blockIdx.x] = t2;
      lp.part_al[blockIdx.x] = low != INT_MAX ? s_al[slot] : 0.0;
      lp.part_bv[blockIdx.x] = low != INT_MAX ? s_bv[slot] : 0;
    }
  }
}

// ---------------------------------------------------------------------------------------
// k_update with compact columns (ld >= kSparseMinLd): the steps and the
// arithmetic of k_update's sparse-column pass at any length of D.  A row's entries on D
// are contiguous in Bc instead of scattered over a row of Binv, and rho comes compact
// (rho_c, formed by the pricing kernel): this wavefront's entries of its first row, of
// rho_c and of the list D are requested in the first round with the control block (the
// first 64 at once, since Bc, rho_c and D hold at least that many entries at these sizes;
// the rest after the scalar load of |D|), so only a_q waits for q.  Workgroup 0 counts the
// changed entries for the byte statistics in one wave, from those registers.  Lane l owns entries
// l, l + 64, ... in ascending order, the fma chain and butterfly of k_update.
template <int B>
__global__ __launch_bounds__(B) void k_update_c(DevLP lp) {
  constexpr int waves = B / 64;
  __shared__ double red_d[2 * waves];
  __shared__ int red_j[2 * waves];
  __shared__ double s_rt[waves * kMaxRowsPerWave];
  __shared__ double s_tau[waves * kMaxRowsPerWave];
  __shared__ int s_row[waves * kMaxRowsPerWave];
  __shared__ double s_al[waves * kMaxRowsPerWave];
  __shared__ int s_bv[waves * kMaxRowsPerWave];
  __shared__ int s_nf;  // some row of this workgroup has a non-finite alpha
  const int m = lp.m, n = lp.n, ld = lp.ld, ld2 = ld / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_nf = 0;  // read after the barriers below
  const int gw = blockIdx.x * waves + wave;
  const int nw = gridDim.x * waves;

  // ---- first round ----
  const Ctrl* ctl = lp.ctrl;
  const int status = ctl->status;
  const int r = ctl->r;
  const int nD = ctl->nD;
  const int cur = ctl->cur;
  const int64_t t = ctl->t;
  const int64_t max_iter = ctl->max_iter;
  const double theta = ctl->theta;
  const int fb = ctl->fb;
  const int bpend = ctl->bpend, q_pend = ctl->q_pend;
  const int pk = min(tid, lp.price_grid - 1);
  double pd0 = lp.part_d[2 * pk], pd1 = lp.part_d[2 * pk + 1];
  int pj0 = lp.part_j[2 * pk], pj1 = lp.part_j[2 * pk + 1];
  const int g0 = min(gw, m - 1);
  double x0 = lp.xB[g0], al00 = lp.alpha0[g0], al10 = lp.alpha1[g0];
  int bv0 = lp.basis[g0];
  if (bpend && g0 == r) bv0 = q_pend;
  double g[kGather], rr[kGather];
  int dj[kGather];
  {
    const double* row = lp.Bc + (size_t)g0 * ld;
#pragma unroll
    for (int u = 0; u < kGather; ++u) {
      const int a = lane + 64 * u;
      g[u] = 0.0;
      rr[u] = 0.0;
      dj[u] = 0;
      if (u == 0 || a < nD) {
        g[u] = row[a];
        rr[u] = lp.rho_c[a];  // (unused when no pivot is pending)
        dj[u] = lp.dlist[a];
      }
    }
  }
  double sd = __builtin_inf();
  int sj = INT_MAX;
  if (lp.mixed) {
    const int w = min(lane, lp.sl_k - 1);
    sd = lp.sl_d[w];
    sj = lp.sl_j[w];
  }
  asm volatile("" ::: "memory");  // compiler-only: every request above is issued first
  if (tid >= lp.price_grid) {
    pd0 = pd1 = __builtin_inf();
    pj0 = pj1 = INT_MAX;
  }

  // Step 4 decision (every workgroup reaches the same q): in the mixed form from the
  // re-priced shortlist (none improving: the fallback verdict), else, and in the mixed
  // form's FP64 pass, from the pricing partials.  As in k_update.
  double da = __builtin_inf(), df = __builtin_inf();
  int ja = INT_MAX, jf = INT_MAX;
  bool from_shortlist = false;
  const bool use_parts = !lp.mixed || fb;
  if (lp.mixed && !fb) {
    if (!(lane < lp.sl_k && sj != INT_MAX && sd < -lp.eps_d)) {
      sd = __builtin_inf();
      sj = INT_MAX;
    }
    wave_lexmin(sd, sj);
    df = sd;
    jf = sj;
    from_shortlist = jf != INT_MAX;
    da = df;
    ja = jf;
  }
  if (use_parts) {
    da = pd0;
    df = pd1;
    ja = pj0;
    jf = pj1;
    for (int k = tid + B; k < lp.price_grid; k += B) {
      const double d0 = lp.part_d[2 * k], d1 = lp.part_d[2 * k + 1];
      const int j0 = lp.part_j[2 * k], j1 = lp.part_j[2 * k + 1];
      if (lex_less(d0, j0, da, ja)) {
        da = d0;
        ja = j0;
      }
      if (lex_less(d1, j1, df, jf)) {
        df = d1;
        jf = j1;
      }
    }
    wave_lexmin(da, ja);
    wave_lexmin(df, jf);
    if (lane == 0) {
      red_d[wave] = da;
      red_j[wave] = ja;
      red_d[waves + wave] = df;
      red_j[waves + wave] = jf;
    }
    __syncthreads();
    da = lane < waves ? red_d[lane] : __builtin_inf();
    ja = lane < waves ? red_j[lane] : INT_MAX;
    df = lane < waves ? red_d[waves + lane] : __builtin_inf();
    jf = lane < waves ? red_j[waves + lane] : INT_MAX;
    wave_lexmin(da, ja);  // every wave reduces the same values: no second exchange needed
    wave_lexmin(df, jf);
  }
  if (status != kStatusRunning) return;
  int verdict = kStatusRunning, q = -1, flags = 0;
  double dq = 0.0;
  if (!use_parts && !from_shortlist) {
    verdict = kVerdictFallback;
  } else if (ja == INT_MAX) {
    verdict = kStatusOptimal;
  } else if (t >= max_iter) {
    verdict = kStatusIterLimit;
  } else if (jf != INT_MAX) {
    q = jf;
    dq = df;
  } else {
    q = ja;
    dq = da;
    flags = kFlagAspiration;
  }
  if (blockIdx.x == 0 && tid == 0) {
    // Only fields no workgroup of this launch reads (as in k_update).
    Ctrl* cw = lp.ctrl;
    // (bpend outlives its pivot: after a stop, a reinversion or the phase switch r is -1)
    if (bpend && r >= 0) lp.basis[r] = q_pend;
    if (cw->gen_q >= 0) {
      lp.gen[cw->gen_q] = cw->gen_val;
      cw->gen_q = -1;
    }
    if (cw->ind_pend >= 0) {  // (no row of this launch has that slack basic)
      lp.inD[cw->ind_pend] = 1;
      cw->ind_pend = -1;
    }
    cw->snap_t = t;
    cw->snap_z = cw->z;
    cw->snap_nD = nD;
    cw->snap_nsb = cw->nsb;
    cw->snap_nL = cw->nL;
    cw->snap_cur = cur;
    if (lp.mixed && !fb) cw->price32_launches += 1;
    if (use_parts) {
      cw->price_cols += n - cw->nsb;
      cw->price_launches += 1;
      if (lp.mixed) cw->full_prices += 1;
    }
    if (r >= 0) cw->wcur ^= 1;  // pricing stored W_new: it is the current top row now
    cw->verdict = verdict;
    cw->q = q;
    cw->dq = dq;
    cw->flags = flags;
    if (flags & kFlagAspiration) cw->n_aspiration += 1;
    if (r >= 0) {
      cw->update_launches += 1;
      cw->update_rows_written += m;
    } else if (q >= 0) {
      cw->update_launches += 1;
    }
  }
  if (r < 0 && q < 0) return;

  // ---- second round: a_q ----
  const double* __restrict__ al_p = cur ? lp.alpha1 : lp.alpha0;  // pending pivot's alpha
  double* __restrict__ al_n = cur ? lp.alpha0 : lp.alpha1;        // FTRAN result for q
  const double eps_p = lp.eps_p, eps_z = lp.eps_z;
  // a_q at this lane's entries of D, gathered from the column (no staging, no barrier); a
  // slack's column is the unit vector e_{q-n}
  const bool q_col = q >= 0 && q < n;
  const double* colq = lp.A + (size_t)(q_col ? q : 0) * ld;
  const int e = q - n;
  double aq[kGather];
#pragma unroll
  for (int u = 0; u < kGather; ++u) {
    const int a = lane + 64 * u;
    aq[u] = 0.0;
    if (q >= 0 && a < nD) aq[u] = q_col ? colq[dj[u]] : (dj[u] == e ? 1.0 : 0.0);
  }
  auto aq_at = [&](int j) { return q_col ? colq[j] : (j == e ? 1.0 : 0.0); };
  // whether the first row's basic variable is a slack outside D (its column of B^-1 is a
  // unit vector): the FTRAN adds its unit term, and the finish needs it for the leaving
  // variable
  int in0 = 1;
  if (gw < m && bv0 >= n) in0 = lp.inD[bv0 - n];
  if (blockIdx.x == 0 && wave == 0) {
    // bytes: the D entries of every row but r read, the changed ones written in every row,
    // one unit lookup (basis, membership, a_q entry) per row
    int nz = 0;
    if (r >= 0) {
#pragma unroll
      for (int u = 0; u < kGather; ++u) nz += (lane + 64 * u < nD && rr[u] != 0.0) ? 1 : 0;
      for (int a = lane + 64 * kGather; a < nD; a += 64) nz += lp.rho_c[a] != 0.0 ? 1 : 0;
    }
    nz = wave_sum_int(nz);
    if (lane == 0) lp.ctrl->update_bytes += 8 * ((int64_t)(m - 1) * nD + (int64_t)m * nz) + 16 * (int64_t)m;
  }
  int c = 0;
  for (int i = gw; i < m; i += nw, ++c) {
    double* row = lp.Bc + (size_t)i * ld;
    double x, alp;
    int bv, in;
    if (c == 0) {
      x = x0;
      alp = cur ? al10 : al00;
      bv = bv0;
      in = in0;
    } else {
      x = lp.xB[i];
      alp = al_p[i];
      bv = (bpend && i == r) ? q_pend : lp.basis[i];
      in = bv >= n ? lp.inD[bv - n] : 1;
#pragma unroll
      for (int u = 0; u < kGather; ++u) {
        const int a = lane + 64 * u;
        if (a < nD) g[u] = row[a];
      }
    }
    const bool isr = i == r;
    const double na = (r >= 0 && !isr) ? -alp : 0.0;
    // the unit column of this row's basic slack, when it is not in D
    const bool unit = q >= 0 && bv >= n && !in;
    const double au = unit ? aq_at(bv - n) : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kGather; ++u) {
      const int a = lane + 64 * u;
      if (a < nD) {
        double val = g[u];
        if (r >= 0) {
          const double rv = rr[u];
          val = isr ? rv : fma(na, rv, val);  // row r := rho (zero wherever rho is zero)
          if (rv != 0.0) row[a] = val;
        }
        if (q >= 0) acc = fma(val, aq[u], acc);
      }
    }
    for (int a = lane + 64 * kGather; a < nD; a += 64) {
      double val = row[a];
      if (r >= 0) {
        const double rv = lp.rho_c[a];
        val = isr ? rv : fma(na, rv, val);
        if (rv != 0.0) row[a] = val;
      }
      if (q >= 0) acc = fma(val, aq_at(lp.dlist[a]), acc);
    }
    if (r >= 0) {
      x = isr ? theta : fma(na, theta, x);
      if (fabs(x) < eps_z) x = 0.0;
      if (lane == 0) lp.xB[i] = x;
    }
    if (q >= 0) {
      acc = wave_sum(acc);
      if (unit) acc += au;
      double rt = __builtin_inf(), tau = __builtin_inf();
      if (acc > eps_p) {
        const double xp = fmax(x, 0.0);
        rt = xp / acc;
        tau = (xp - lp.eps_t) / acc;
        tau -= 1e-12 * (fabs(tau) + 1.0);
      }
      if (lane == 0) {
        al_n[i] = acc;
        s_rt[wave * kMaxRowsPerWave + c] = rt;
        s_tau[wave * kMaxRowsPerWave + c] = tau;
        s_row[wave * kMaxRowsPerWave + c] = acc > eps_p ? i : INT_MAX;  // INT_MAX: not a candidate
        if (!isfinite(acc)) s_nf = 1;
        s_al[wave * kMaxRowsPerWave + c] = acc;
        s_bv[wave * kMaxRowsPerWave + c] = 2 * bv + ((bv < n || in) ? 1 : 0);
      }
    }
  }
  if (q < 0) return;
  // Workgroup partial of Step 6 (as k_update).
  for (int k = c; k < kMaxRowsPerWave; ++k)
    if (lane == 0) {
      s_rt[wave * kMaxRowsPerWave + k] = __builtin_inf();
      s_tau[wave * kMaxRowsPerWave + k] = __builtin_inf();
      s_row[wave * kMaxRowsPerWave + k] = INT_MAX;
    }
  __syncthreads();
  if (wave == 0) {
    constexpr int slots = waves * kMaxRowsPerWave;
    double th = __builtin_inf(), t1 = __builtin_inf(), t2 = __builtin_inf();
    int low = INT_MAX, slot = 0;
    for (int k = lane; k < slots; k += 64) {
      if (lex_less(s_rt[k], s_row[k], th, low)) {
        th = s_rt[k];
        low = s_row[k];
        slot = k;
      }
      const double tk = s_tau[k];
      if (tk < t1) {
        t2 = t1;
        t1 = tk;
      } else if (tk < t2) {
        t2 = tk;
      }
    }
    wave_lexmin_payload(th, low, slot);
    wave_two_smallest(t1, t2);
    if (lane == 0) {
      lp.part_th[blockIdx.x] = s_nf ? -__builtin_inf() : th;
      lp.part_low[blockIdx.x] = s_nf ? -1 : low;
      lp.part_t1[blockIdx.x] = t1;
      lp.part_t2[blockIdx.x] = t2;
      lp.part_al[blockIdx.x] = low != INT_MAX ? s_al[slot] : 0.0;
      lp.part_bv[blockIdx.x] = low != INT_MAX ? s_bv[slot] : 0;
    }
  }
}

// Compact columns on request (no pivot pending): Binv's columns in D from Bc (each thread
// one row entry), and Bc from Binv and the list D.  Columns of Bc from |D| on must be zero:
// the rebuild clears those below nd_prev, the length of D before the step that changed it
// (the ones beyond were zero already).
__global__ void k_materialize(DevLP lp) {
  const int nD = lp.ctrl->nD, ld = lp.ld;
  const size_t total = (size_t)lp.m * nD;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < total; k += stride) {
    const size_t i = k / nD, a = k - i * nD;
    lp.Binv[i * ld + lp.dlist[a]] = lp.Bc[i * ld + a];
  }
}
__global__ void k_rebuild_compact(DevLP lp, int nd_prev) {
  const int nD = lp.ctrl->nD, ld = lp.ld;
  const int w = max(nD, nd_prev);
  const size_t total = (size_t)lp.m * w;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < total; k += stride) {
    const size_t i = k / w, a = k - i * w;
    lp.Bc[i * ld + a] = (int)a < nD ? lp.Binv[i * ld + lp.dlist[a]] : 0.0;
  }
}

// ---------------------------------------------------------------------------------------
// k_update for rows too long for k_update's staging of the whole of rho and a_q (16.5 ld
// bytes of LDS, so above ld = 9792).  The same steps and the same arithmetic, staged
// differently: in sparse-column mode only the list D and rho, a_q at its entries (20 bytes
// per entry, ld / 8 entries at most); in dense mode rho and a_q in chunks of kWideChunk2
// element pairs, each wavefront carrying the running dot products of its rows from chunk
// to chunk.  Lane l still owns pairs l, l + 64, ... of a row in ascending order (chunks are
// multiples of 64 pairs) and D entries l, l + 64, ..., so every alpha_i is the same fma
// chain and butterfly as in k_update.
constexpr int kWideChunk2 = 2048;

template <int B>
__global__ __launch_bounds__(B) void k_update_wide(DevLP lp) {
  constexpr int waves = B / 64;
  constexpr int R = kMaxRowsPerWave;
  extern __shared__ double2 wsm[];
  __shared__ double red_d[2 * waves];
  __shared__ int red_j[2 * waves];
  __shared__ double s_rt[waves * R];
  __shared__ double s_tau[waves * R];
  __shared__ int s_row[waves * R];
  __shared__ double s_al[waves * R];
  __shared__ int s_bv[waves * R];
  __shared__ int s_nf;
  const int n = lp.n, ld = lp.ld, ld2 = ld / 2;
  const int lo = lp.row_lo, hi = lp.row_hi;
  const bool first_panel = lo == 0;
  const int m = lp.m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_nf = 0;
  const int gw = blockIdx.x * waves + wave;
  const int nw = gridDim.x * waves;
  const int i0 = lo + gw;

  const Ctrl* ctl = lp.ctrl;
  const int status = ctl->status;
  const int r = ctl->r;
  const int nD = ctl->nD;
  const int cur = ctl->cur;
  const int64_t t = ctl->t;
  const int64_t max_iter = ctl->max_iter;
  const double theta = ctl->theta;
  const int fb = ctl->fb;

  // Step 4 decision, as in k_update.
  double da = __builtin_inf(), df = __builtin_inf();
  int ja = INT_MAX, jf = INT_MAX;
  bool from_shortlist = false;
  const bool use_parts = !lp.mixed || fb;
  if (lp.mixed && !fb) {
    double sd = __builtin_inf();
    int sj = INT_MAX;
    const int w = min(lane, lp.sl_k - 1);
    sd = lp.sl_d[w];
    sj = lp.sl_j[w];
    if (!(lane < lp.sl_k && sj != INT_MAX && sd < -lp.eps_d)) {
      sd = __builtin_inf();
      sj = INT_MAX;
    }
    wave_lexmin(sd, sj);
    df = sd;
    jf = sj;
    from_shortlist = jf != INT_MAX;
    da = df;
    ja = jf;
  }
  if (use_parts) {
    for (int k = tid; k < lp.price_grid; k += B) {
      const double d0 = lp.part_d[2 * k], d1 = lp.part_d[2 * k + 1];
      const int j0 = lp.part_j[2 * k], j1 = lp.part_j[2 * k + 1];
      if (lex_less(d0, j0, da, ja)) {
        da = d0;
        ja = j0;
      }
      if (lex_less(d1, j1, df, jf)) {
        df = d1;
        jf = j1;
      }
    }
    wave_lexmin(da, ja);
    wave_lexmin(df, jf);
    if (lane == 0) {
      red_d[wave] = da;
      red_j[wave] = ja;
      red_d[waves + wave] = df;
      red_j[waves + wave] = jf;
    }
    __syncthreads();
    da = lane < waves ? red_d[lane] : __builtin_inf();
    ja = lane < waves ? red_j[lane] : INT_MAX;
    df = lane < waves ? red_d[waves + lane] : __builtin_inf();
    jf = lane < waves ? red_j[waves + lane] : INT_MAX;
    wave_lexmin(da, ja);
    wave_lexmin(df, jf);
  }
  __syncthreads();
  if (status != kStatusRunning) return;
  const bool sparse = sparse_columns(nD, ld);
  int verdict = kStatusRunning, q = -1, flags = 0;
  double dq = 0.0;
  if (!use_parts && !from_shortlist) {
    verdict = kVerdictFallback;
  } else if (ja == INT_MAX) {
    verdict = kStatusOptimal;
  } else if (t >= max_iter) {
    verdict = kStatusIterLimit;
  } else if (jf != INT_MAX) {
    q = jf;
    dq = df;
  } else {
    q = ja;
    dq = da;
    flags = kFlagAspiration;
  }
  if (blockIdx.x == 0 && tid == 0 && first_panel) {
    Ctrl* cw = lp.ctrl;
    if (lp.mixed && !fb) cw->price32_launches += 1;
    if (use_parts) {
      cw->price_cols += n - cw->nsb;
      cw->price_launches += 1;
      if (lp.mixed) cw->full_prices += 1;
    }
    if (r >= 0) cw->wcur ^= 1;
    cw->verdict = verdict;
    cw->q = q;
    cw->dq = dq;
    cw->flags = flags;
    if (flags & kFlagAspiration) cw->n_aspiration += 1;
    if (r >= 0) {
      cw->update_launches += 1;
      cw->update_rows_written += m;
    } else if (q >= 0) {
      cw->update_launches += 1;
    }
    if (!sparse && (r >= 0 || q >= 0)) {
      cw->update_bytes += 8 * (int64_t)m * m;
      if (r >= 0) cw->update_bytes += 16 * ((int64_t)(m - 1) * cw->rho_nz2 + ld / 2);
    }
  }
  if (r < 0 && q < 0) return;

  const double* __restrict__ al_p = cur ? lp.alpha1 : lp.alpha0;
  double* __restrict__ al_n = cur ? lp.alpha0 : lp.alpha1;
  const double eps_p = lp.eps_p, eps_z = lp.eps_z;
  const bool q_col = q >= 0 && q < n;
  const int qs = q >= n ? q - n : -1;  // a slack entering: a_q = e_qs
  const double* __restrict__ aq = lp.A + (size_t)(q_col ? q : 0) * ld;
  // This wavefront's rows and their state.
  double xr[R], nar[R], acc[R];
  int bvr[R], inr[R];
  int nrows = 0;
#pragma unroll
  for (int c = 0; c < R; ++c) {
    const int i = i0 + c * nw;
    acc[c] = 0.0;
    if (i < hi) {
      nrows = c + 1;
      xr[c] = lp.xB[i];
      const int bv = lp.basis[i];
      bvr[c] = bv;
      inr[c] = bv >= n ? lp.inD[bv - n] : 1;
      nar[c] = (r >= 0 && i != r) ? -al_p[i] : 0.0;
    }
  }
  if (sparse) {
    const int dcap = ld / 8;
    double* s_rD = reinterpret_cast<double*>(wsm);
    double* s_aD = s_rD + dcap;
    int* s_dl = reinterpret_cast<int*>(s_aD + dcap);
    int nz = 0;
    for (int k = tid; k < nD; k += B) {
      const int j = lp.dlist[k];
      s_dl[k] = j;
      const double rr = r >= 0 ? lp.rho[j] : 0.0;
      s_rD[k] = rr;
      nz += rr != 0.0 ? 1 : 0;
      s_aD[k] = q_col ? aq[j] : (j == qs ? 1.0 : 0.0);
    }
    if (blockIdx.x == 0 && first_panel) {
      nz = block_sum_int<B>(nz, red_j);
      if (tid == 0) lp.ctrl->update_bytes += 8 * ((int64_t)(m - 1) * nD + (int64_t)m * nz) + 16 * (int64_t)m;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < R; ++c) {
      if (c >= nrows) break;
      const int i = i0 + c * nw;
      double* row = lp.Binv + (size_t)(i - lo) * ld;
      const bool isr = i == r;
      for (int a = lane; a < nD; a += 64) {
        const int j = s_dl[a];
        double val = row[j];
        if (r >= 0) {
          const double rr = s_rD[a];
          val = isr ? rr : fma(nar[c], rr, val);
          if (rr != 0.0) row[j] = val;
        }
        if (q >= 0) acc[c] = fma(val, s_aD[a], acc[c]);
      }
    }
  } else {
    double2* s_rho = wsm;
    double2* s_a = wsm + kWideChunk2;
    const double2* rho2 = reinterpret_cast<const double2*>(lp.rho);
    const double2* aq2 = reinterpret_cast<const double2*>(aq);
    for (int c0 = 0; c0 < ld2; c0 += kWideChunk2) {
      const int cn = min(kWideChunk2, ld2 - c0);
      __syncthreads();  // the previous chunk has been used
      for (int k = tid; k < cn; k += B) {
        if (r >= 0) s_rho[k] = rho2[c0 + k];
        if (q >= 0) {
          const int e = 2 * (c0 + k);
          s_a[k] = q_col ? aq2[c0 + k] : make_double2(e == qs ? 1.0 : 0.0, e + 1 == qs ? 1.0 : 0.0);
        }
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (c >= nrows) break;
        const int i = i0 + c * nw;
        double2* row = reinterpret_cast<double2*>(lp.Binv + (size_t)(i - lo) * ld) + c0;
        const bool isr = i == r;
        for (int k = lane; k < cn; k += 64) {
          double2 v = row[k];
          if (r >= 0) {
            const double2 rr = s_rho[k];
            if (isr) {
              v = rr;
              row[k] = v;
            } else {
              v.x = fma(nar[c], rr.x, v.x);
              v.y = fma(nar[c], rr.y, v.y);
              if (rr.x != 0.0 || rr.y != 0.0) row[k] = v;
            }
          }
          if (q >= 0) {
            const double2 w = s_a[k];
            acc[c] = fma(v.x, w.x, acc[c]);
            acc[c] = fma(v.y, w.y, acc[c]);
          }
        }
      }
    }
  }
  // x_B, alpha and the per-row part of Step 6, as in k_update.
  int c = 0;
#pragma unroll
  for (int cc = 0; cc < R; ++cc) {
    if (cc >= nrows) break;
    c = cc + 1;
    const int i = i0 + cc * nw;
    const bool isr = i == r;
    double x = xr[cc];
    if (r >= 0) {
      x = isr ? theta : fma(nar[cc], theta, x);
      if (fabs(x) < eps_z) x = 0.0;
      if (lane == 0) lp.xB[i] = x;
    }
    if (q >= 0) {
      double a = wave_sum(acc[cc]);
      const int bv = bvr[cc];
      if (sparse && bv >= n && !inr[cc]) a += q_col ? aq[bv - n] : (bv - n == qs ? 1.0 : 0.0);
      double rt = __builtin_inf(), tau = __builtin_inf();
      if (a > eps_p) {
        const double xp = fmax(x, 0.0);
        rt = xp / a;
        tau = (xp - lp.eps_t) / a;
        tau -= 1e-12 * (fabs(tau) + 1.0);
      }
      if (lane == 0) {
        al_n[i] = a;
        s_rt[wave * R + cc] = rt;
        s_tau[wave * R + cc] = tau;
        s_row[wave * R + cc] = a > eps_p ? i : INT_MAX;
        if (!isfinite(a)) s_nf = 1;
        s_al[wave * R + cc] = a;
        s_bv[wave * R + cc] = 2 * bv + ((bv < n || inr[cc]) ? 1 : 0);
      }
    }
  }
  if (q < 0) return;
  for (int k = c; k < R; ++k)
    if (lane == 0) {
      s_rt[wave * R + k] = __builtin_inf();
      s_tau[wave * R + k] = __builtin_inf();
      s_row[wave * R + k] = INT_MAX;
    }
  __syncthreads();
  if (wave == 0) {
    constexpr int slots = waves * R;
    double th = __builtin_inf(), t1 = __builtin_inf(), t2 = __builtin_inf();
    int low = INT_MAX, slot = 0;
    for (int k = lane; k < slots; k += 64) {
      if (lex_less(s_rt[k], s_row[k], th, low)) {
        th = s_rt[k];
        low = s_row[k];
        slot = k;
      }
      const double tk = s_tau[k];
      if (tk < t1) {
        t2 = t1;
        t1 = tk;
      } else if (tk < t2) {
        t2 = tk;
      }
    }
    wave_lexmin_payload(th, low, slot);
    wave_two_smallest(t1, t2);
    if (lane == 0) {
      lp.part_th[blockIdx.x] = s_nf ? -__builtin_inf() : th;
      lp.part_low[blockIdx.x] = s_nf ? -1 : low;
      lp.part_t1[blockIdx.x] = t1;
      lp.part_t2[blockIdx.x] = t2;
      lp.part_al[blockIdx.x] = low != INT_MAX ? s_al[slot] : 0.0;
      lp.part_bv[blockIdx.x] = low != INT_MAX ? s_bv[slot] : 0;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Step 6 finish and the scalar part of Step 8.  Every k_update workgroup left its minimum
// ratio (with the lowest row attaining it, that row's alpha and basic variable) and the two
// smallest tie thresholds of its rows; x_B and alpha of this iteration are in memory.
//
// finish_step is run by the one workgroup of k_finish, and by every workgroup of
// k_price_fin, the kernel that fuses it with the next pricing pass.  Each workgroup takes
// the same decision from the same inputs; one thread of workgroup 0 commits it.  In the
// fused kernel the other workgroups still read while that thread writes, so there the
// commit leaves alone what they read: the inputs come from the snapshot k_update took
// (FinishIn), basis[r] and the tabu list's generation bump are left for the next k_update
// to apply, and the pricing part patches its own view of pos and tabu_until.
// Rows of B^-1 per thread per round in the tie scans below, every load of a round issued
// before any test (a loop over the rows waits for each row's loads in turn); more per round
// spill registers in k_price_fin, where the first batch of A' is held across the finish.
constexpr int kTieRound = 2;
// Entries of the leaving-side list per thread per round in its scan (the same reason; the
// list grows by one entry per tied pivot).
constexpr int kListRound = 4;
template <int B, bool FUSED>
__device__ FinishOut finish_step(const DevLP& lp, const FinishIn& in, double pth, double pt1, double pt2, double pal,
                                 int plow, int pbv) {
  __shared__ double red_d[B / 64 + 8];
  __shared__ int red_j[2 * (B / 64) + 8];
  __shared__ double s_pick_al;
  __shared__ int s_pick[3];
  Ctrl* ctl = lp.ctrl;
  const int m = lp.m, tid = threadIdx.x, nparts = lp.update_grid;
  const bool writer = tid == 0 && (!FUSED || blockIdx.x == 0);
  const int verdict = in.verdict, q = in.q, cur = in.cur, flags0 = in.flags0, nD0 = in.nD0, nsb0 = in.nsb0;
  const int64_t t = in.t;
  const double dq = in.dq, z0 = in.z0;
  FinishOut out{0, -1, -1, 1, 0.0};
  if (tid >= nparts) {
    pth = pt1 = pt2 = __builtin_inf();
    plow = INT_MAX;
  }
  if (verdict < 0) return out;  // k_update did not run
  if (!FUSED && writer) ctl->fb = verdict == kVerdictFallback ? 1 : 0;
  if (verdict == kVerdictFallback) {  // no pivot; k_update applied the pending one
    if (writer) {
      ctl->verdict = -1;
      ctl->r = -1;
      ctl->q = -1;
      ctl->n_fallback += 1;
    }
    return out;
  }
  if (verdict != kStatusRunning) {  // OPTIMAL or ITER_LIMIT; k_update applied the pending pivot
    if (writer) {
      ctl->status = verdict;
      ctl->r = -1;
      if (!FUSED) {
        ctl->verdict = -1;
        ctl->q = -1;
      }
    }
    return out;
  }

  const double* al = cur ? lp.alpha0 : lp.alpha1;  // FTRAN result of this iteration
  // (minimum ratio, lowest candidate row): row INT_MAX means no candidate row, and
  // (-inf, -1) a non-finite alpha somewhere.
  double th = pth;
  int lowc = plow;
  for (int k = tid + B; k < nparts; k += B) {
    const double d = lp.part_th[k];
    const int j = lp.part_low[k];
    if (lex_less(d, j, th, lowc)) {
      th = d;
      lowc = j;
    }
  }
  block_lexmin<B>(th, lowc, red_d, red_j);
  const bool nonfinite = th == -__builtin_inf() || (lowc != INT_MAX && !isfinite(th));
  if (nonfinite || lowc == INT_MAX) {
    if (writer) {
      if (nonfinite) {
        ctl->status = kStatusNumerical;
      } else {  // Step 5: Y_k <= 0
        ctl->status = kStatusUnbounded;
        ctl->ray = q;
      }
      ctl->r = -1;
      if (!FUSED) {
        ctl->verdict = -1;
        ctl->q = -1;
      }
    }
    return out;
  }
  // A row is tied when it reaches zero (within eps_t) at the step th; exact test below.
  const double eps_p = lp.eps_p, eps_t = lp.eps_t;
  // Fast path: one workgroup may hold tied rows, and only one of its rows may.  Its
  // partial then names the pivot row, with that row's alpha and basic variable.
  int ncand = 0, cand = INT_MAX;
  if (tid < nparts && pt1 <= th) {
    ncand = 1;
    cand = tid;
  }
  for (int k = tid + B; k < nparts; k += B)
    if (lp.part_t1[k] <= th) {
      ++ncand;
      cand = min(cand, k);
    }
  block_sum_min_int<B>(ncand, cand, red_j);
  bool fast = false;
  if (ncand == 1) {
    if (cand < B) {
      if (tid == cand) {
        s_pick[0] = pt2 > th ? 1 : 0;
        s_pick[1] = plow;
        s_pick[2] = pbv;
        s_pick_al = pal;
      }
    } else if (tid == 0) {
      s_pick[0] = lp.part_t2[cand] > th ? 1 : 0;
      s_pick[1] = lp.part_low[cand];
      s_pick[2] = lp.part_bv[cand];
      s_pick_al = lp.part_al[cand];
    }
    __syncthreads();
    fast = s_pick[0] != 0;
  }
  int cnt, low;
  if (fast) {
    cnt = 1;
    low = s_pick[1];
  } else {
    cnt = 0;
    low = INT_MAX;
    for (int i0 = tid; i0 < m; i0 += kTieRound * B) {
      double a[kTieRound], x[kTieRound];
#pragma unroll
      for (int u = 0; u < kTieRound; ++u) {
        const int i = i0 + u * B;
        a[u] = 0.0;
        x[u] = 0.0;
        if (i < m) {
          a[u] = al[i];
          x[u] = lp.xB[i];
        }
      }
#pragma unroll
      for (int u = 0; u < kTieRound; ++u) {
        const int i = i0 + u * B;
        if (i < m && a[u] > eps_p && fma(-a[u], th, fmax(x[u], 0.0)) <= eps_t) {
          ++cnt;
          low = min(low, i);
        }
      }
    }
    block_sum_min_int<B>(cnt, low, red_j);
  }
  int r = low;
  int flags = flags0;
  if (cnt >= 2) {
    flags |= kFlagTie;
    if (lp.use_llist) {
      // (every workgroup of the fused kernel stamps the same entries with the same value)
      const int stamp = (int)t + 1;
      const int g = lp.gen[q];
      const int nL = in.nL;
      for (int k0 = tid; k0 < nL; k0 += kListRound * B) {
        int lq[kListRound], lg[kListRound];
#pragma unroll
        for (int u = 0; u < kListRound; ++u) {
          const int k = k0 + u * B;
          lq[u] = -1;
          lg[u] = 0;
          if (k < nL) {
            lq[u] = lp.Lq[k];
            lg[u] = lp.Lgen[k];
          }
        }
#pragma unroll
        for (int u = 0; u < kListRound; ++u) {
          const int k = k0 + u * B;
          if (k < nL && lq[u] == q && lg[u] == g) lp.excl[lp.Ll[k]] = stamp;
        }
      }
      __syncthreads();
      int fl = INT_MAX;
      for (int i0 = tid; i0 < m; i0 += kTieRound * B) {
        double a[kTieRound], x[kTieRound];
        int bv[kTieRound];
#pragma unroll
        for (int u = 0; u < kTieRound; ++u) {
          const int i = i0 + u * B;
          a[u] = 0.0;
          x[u] = 0.0;
          bv[u] = 0;
          if (i < m) {
            a[u] = al[i];
            x[u] = lp.xB[i];
            bv[u] = lp.basis[i];
          }
        }
#pragma unroll
        for (int u = 0; u < kTieRound; ++u) {
          const int i = i0 + u * B;
          if (i < m && a[u] > eps_p && fma(-a[u], th, fmax(x[u], 0.0)) <= eps_t && lp.excl[bv[u]] != stamp)
            fl = min(fl, i);
        }
      }
      fl = block_min_int<B>(fl, red_j);
      int gnew = g;
      if (fl == INT_MAX) {
        flags |= kFlagLClear;
        gnew = g + 1;
      } else {
        r = fl;
      }
      if (writer) {
        if (gnew != g) {
          if (FUSED) {
            ctl->gen_q = q;  // applied by the next k_update (gen[q] is read above)
            ctl->gen_val = gnew;
          } else {
            lp.gen[q] = gnew;
          }
        }
        if (nL < lp.Lcap) {
          lp.Lq[nL] = q;
          lp.Ll[nL] = lp.basis[r];
          lp.Lgen[nL] = gnew;
          ctl->nL = nL + 1;
        }
      }
    }
  }
  // Step 8 pivots on row r with the step th.
  int leave, kept;  // kept: the leaving variable is structural or its slack is in D already
  double ar;
  if (fast) {
    leave = s_pick[2] >> 1;
    kept = s_pick[2] & 1;
    ar = s_pick_al;
  } else {
    leave = lp.basis[r];
    kept = leave < lp.n || lp.inD[leave - lp.n];
    ar = al[r];
  }
  if (writer) {
    const double thr = th;
    if (thr == 0.0) flags |= kFlagDegenerate;
    if (lp.tenure > 0) lp.tabu_until[leave] = (int)(t + lp.tenure);
    if (!kept) {  // its column of B^-1 stops being a unit vector
      if (FUSED) {
        ctl->ind_pend = leave - lp.n;  // set by the next k_update (inD is read above)
      } else {
        lp.inD[leave - lp.n] = 1;
      }
      lp.dlist[nD0] = leave - lp.n;
      ctl->nD = nD0 + 1;
    }
    ctl->dapp = kept ? -1 : nD0;
    ctl->z = fma(dq, thr, z0);
    if (FUSED) {
      ctl->q_pend = q;  // basis[r] = q, applied by the next k_update
      ctl->bpend = 1;
    } else {
      lp.basis[r] = q;
      ctl->bpend = 0;
    }
    lp.pos[q] = r;
    lp.pos[leave] = (lp.art && leave >= lp.n && lp.art[leave - lp.n]) ? kPosBarred : -1;
    ctl->nsb = nsb0 + (q < lp.n ? 1 : 0) - (leave < lp.n ? 1 : 0);
    if (t < lp.log_cap) {
      lp.log_enter[t] = q;
      lp.log_row[t] = r;
      lp.log_leave[t] = leave;
      lp.log_flags[t] = flags;
    }
    if (flags & kFlagTie) ctl->n_tie += 1;
    if (flags & kFlagLClear) ctl->n_lclear += 1;
    if (flags & kFlagDegenerate) ctl->n_degenerate += 1;
    ctl->t = t + 1;
    ctl->r = r;        // pending: rows of B^-1 and x_B are pivoted by the next k_update,
    ctl->theta = thr;  // the top row by the next pricing kernel
    ctl->pdq = dq;
    ctl->ar = ar;
    ctl->cur = cur ^ 1;
    if (!FUSED) {
      ctl->q = -1;
      ctl->flags = 0;
      ctl->verdict = -1;
    }
  }
  out.pivot = 1;
  out.r = r;
  out.leave = leave;
  out.kept = kept;
  out.ar = ar;
  return out;
}

__global__ __launch_bounds__(kFinishBlock) void k_finish(DevLP lp) {
  const Ctrl* ctl = lp.ctrl;
  const int tid = threadIdx.x, nparts = lp.update_grid;
  // One round of requests: the control block and the first partial of every thread.
  FinishIn in;
  const int status = ctl->status;
  in.verdict = ctl->verdict;
  in.q = ctl->q;
  in.cur = ctl->cur;
  in.t = ctl->t;
  in.flags0 = ctl->flags;
  in.dq = ctl->dq;
  in.z0 = ctl->z;
  in.nD0 = ctl->nD;
  in.nsb0 = ctl->nsb;
  in.nL = ctl->nL;
  const int pk = min(tid, nparts - 1);  // clamped, not guarded: no load waits behind a branch
  const double pth = lp.part_th[pk], pt1 = lp.part_t1[pk], pt2 = lp.part_t2[pk], pal = lp.part_al[pk];
  const int plow = lp.part_low[pk], pbv = lp.part_bv[pk];
  asm volatile("" ::: "memory");  // compiler-only: all of the above is requested first
  if (status != kStatusRunning) return;
  finish_step<kFinishBlock, false>(lp, in, pth, pt1, pt2, pal, plow, pbv);
}

// ---------------------------------------------------------------------------------------
// Out-of-core panel mode: after the ratio test, row r of B^-1 (the rows already updated by
// this iteration's panel pass) is copied into `row` for the next pricing kernel, from the
// device-resident last panel (rows res_lo..) or from the pinned host copy.
__global__ void k_fetch_row(const Ctrl* __restrict__ ctl, const double* __restrict__ host, const double* __restrict__ res,
                            int res_lo, int ld, double* __restrict__ row) {
  const int r = ctl->r;
  if (r < 0) return;
  const double* src = r >= res_lo ? res + (size_t)(r - res_lo) * ld : host + (size_t)r * ld;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ld; k += gridDim.x * blockDim.x) row[k] = src[k];
}

// ---------------------------------------------------------------------------------------
// Helpers of the entry point that allocates nothing (its buffers live in a fixed array).

// *flag = 0 (a kernel rather than a memset, so that a captured stream holds no memset node).
__global__ void k_clear_flag(int32_t* flag) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
}

// Copies the caller's A' (m x n, column-major, lda = m) into the padded ld x n layout with
// zero padding, and b, c into b0, c0; sets bit 1 of *flag for a non-finite entry of A', b
// or c, bit 2 for some b_i < 0.
__global__ void k_pack_lp(double* __restrict__ dA, int ld, const double* __restrict__ A, int m, int n,
                          double* __restrict__ b0, const double* __restrict__ b, double* __restrict__ c0,
                          const double* __restrict__ c, int32_t* flag) {
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  int bad = 0;
  const size_t total = (size_t)ld * n;
  for (size_t k = tid; k < total; k += stride) {
    const size_t j = k / ld, i = k - j * ld;
    double v = 0.0;
    if (i < (size_t)m) {
      v = A[j * m + i];
      bad |= isfinite(v) ? 0 : 1;
    }
    dA[k] = v;
  }
  for (size_t i = tid; i < (size_t)m; i += stride) {
    const double v = b[i];
    b0[i] = v;
    bad |= isfinite(v) ? 0 : 1;
    bad |= v < 0.0 ? 2 : 0;
  }
  for (size_t j = tid; j < (size_t)n; j += stride) {
    const double v = c[j];
    c0[j] = v;
    bad |= isfinite(v) ? 0 : 1;
  }
  if (bad) atomicOr(flag, bad);
}

// Adds the hash terms of x[0..nx) (indices base + k), y and z (indices following x's) to *out.
__global__ void k_hash(const double* __restrict__ x, size_t nx, uint64_t base, const double* __restrict__ y, size_t ny,
                       const double* __restrict__ z, size_t nz, unsigned long long* out) {
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  uint64_t h = 0;
  for (size_t k = tid; k < nx; k += stride) h += hash_word(__double_as_longlong(x[k]), base + k);
  for (size_t k = tid; k < ny; k += stride) h += hash_word(__double_as_longlong(y[k]), base + nx + k);
  for (size_t k = tid; k < nz; k += stride) h += hash_word(__double_as_longlong(z[k]), base + nx + ny + k);
  if (h) atomicAdd(out, (unsigned long long)h);
}

__global__ void k_clear_u64(unsigned long long* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *out = 0;
}

// The pivot limit and the RUNNING status of a fresh solve.
__global__ void k_arm(Ctrl* ctl, int64_t max_iter) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->max_iter = max_iter;
    ctl->status = kStatusRunning;
  }
}

// x (n), y = ysign * W (m) and the objective sum_j c_j x_j over structural basics in
// ascending j (the order of lp_get_solution); any pointer may be null.
__global__ void k_solution(DevLP lp, const double* __restrict__ c, double ysign, double* __restrict__ x,
                           double* __restrict__ y, double* __restrict__ objective) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  const double* W = lp.ctrl->wcur ? lp.W1 : lp.W0;
  if (x)
    for (int j = tid; j < lp.n; j += stride) {
      const int r = lp.pos[j];
      x[j] = r >= 0 ? lp.xB[r] : 0.0;
    }
  if (y)
    for (int i = tid; i < lp.m; i += stride) y[i] = ysign * W[i];
  if (objective && tid == 0) {
    double s = 0.0;
    for (int j = 0; j < lp.n; ++j) {
      const int r = lp.pos[j];
      if (r >= 0) s = __dadd_rn(s, __dmul_rn(c[j], lp.xB[r]));
    }
    *objective = s;
  }
}

// Sets *flag when some |x_k| exceeds bound or is NaN.
__global__ void k_check_finite(const double* __restrict__ x, int64_t count, double bound, int32_t* flag) {
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (size_t k = tid; k < (size_t)count; k += stride) bad |= !(fabs(x[k]) <= bound);
  if (bad) *flag = 1;
}

// ---------------------------------------------------------------------------------------
const void* price_kernel(bool nt) {
  return nt ? reinterpret_cast<const void*>(&k_price<true>) : reinterpret_cast<const void*>(&k_price<false>);
}
const void* price_fin_kernel(bool nt) {
  return nt ? reinterpret_cast<const void*>(&k_price_fin<true>) : reinterpret_cast<const void*>(&k_price_fin<false>);
}
bool price_nt(int ld, int n) { return sizeof(double) * (size_t)ld * (size_t)n > kLastLevelCacheBytes; }
// k_update's workgroup size for a row stride ld: kUpdateBlock threads, or twice that where
// the staging in LDS admits only one such workgroup per CU and one of the larger ones
// fits (it keeps twice the wavefronts in flight); -kUpdateBlock: k_update_wide, for rows
// whose staging does not fit at all.
size_t wide_lds_bytes(int ld) {
  return std::max<size_t>(2 * sizeof(double2) * (size_t)kWideChunk2, (2 * sizeof(double) + sizeof(int)) * (size_t)(ld / 8));
}
int update_block(int ld) {
  const int lds = (int)update_lds_bytes(ld);
  int small = 0, large = 0;
  const void* fs = reinterpret_cast<const void*>(&k_update<kUpdateBlock>);
  const void* fl = reinterpret_cast<const void*>(&k_update<2 * kUpdateBlock>);
  if (ld > kUpdateStageMaxLd) return 0;  // rows beyond LP_MAX_ROWS: not launched (see k_update_wide)
  if (hipFuncSetAttribute(fs, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&small, k_update<kUpdateBlock>, kUpdateBlock, lds) != hipSuccess) {
    (void)hipGetLastError();  // reported by the caller's own occupancy query
    return kUpdateBlock;
  }
  if (small >= 2) return kUpdateBlock;
  // The larger workgroup has more static LDS: near the largest ld it may not fit at all,
  // and a refused attribute would otherwise stay as the runtime's last error.
  if (hipFuncSetAttribute(fl, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&large, k_update<2 * kUpdateBlock>, 2 * kUpdateBlock, lds) !=
          hipSuccess) {
    (void)hipGetLastError();
    return kUpdateBlock;
  }
  return large >= 1 ? 2 * kUpdateBlock : kUpdateBlock;
}
const void* update_kernel_for_block(int block) {
  return block == kUpdateBlock ? reinterpret_cast<const void*>(&k_update<kUpdateBlock>)
         : block > 0           ? reinterpret_cast<const void*>(&k_update<2 * kUpdateBlock>)
                               : reinterpret_cast<const void*>(&k_update_wide<kUpdateBlock>);
}
const void* update_kernel(int ld) { return update_kernel_for_block(update_block(ld)); }
const void* update_kernel_for(const DevLP& lp) {
  return lp.cmode ? reinterpret_cast<const void*>(&k_update_c<kUpdateBlock>) : update_kernel_for_block(lp.upd_block);
}
const void* finish_kernel() { return reinterpret_cast<const void*>(&k_finish); }

size_t price_lds_bytes(int ld) { return sizeof(double) * (size_t)ld; }
// rho and a_q (ld doubles each) and, where sparse mode is possible, list D (ld/8 ints)
size_t update_lds_bytes(int ld) {
  return 2 * sizeof(double) * (size_t)ld + (ld >= kSparseMinLd ? sizeof(int) * (size_t)(ld / 8) : 0);
}
size_t update_lds_for_block(int block, int ld) { return block > 0 ? update_lds_bytes(ld) : wide_lds_bytes(ld); }
// k_update_c stages nothing in dynamic LDS
size_t compact_lds_bytes(int) { return 0; }

hipError_t kernel_occupancy(int* price_per_cu, int* update_per_cu, int ld, bool cmode) {
  hipError_t e = hipSuccess;
  for (const bool nt : {false, true}) {
    e = hipFuncSetAttribute(price_kernel(nt), hipFuncAttributeMaxDynamicSharedMemorySize, (int)price_lds_bytes(ld));
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(price_fin_kernel(nt), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)price_lds_bytes(ld));
    if (e != hipSuccess) return e;
  }
  const int blk = update_block(ld);
  if (blk == 0) return hipErrorInvalidValue;
  const int lds = (int)update_lds_for_block(blk, ld);
  e = hipFuncSetAttribute(update_kernel_for_block(blk), hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  if (cmode) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_update_c<kUpdateBlock>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)compact_lds_bytes(ld));
    if (e != hipSuccess) return e;
  }
  // The pricing grid serves every pricing kernel: size it for the one that fits fewest.
  int occ[4] = {0, 0, 0, 0};
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[0], k_price<false>, kPriceBlock, price_lds_bytes(ld));
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[1], k_price<true>, kPriceBlock, price_lds_bytes(ld));
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[2], k_price_fin<false>, kPriceBlock, price_lds_bytes(ld));
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[3], k_price_fin<true>, kPriceBlock, price_lds_bytes(ld));
  if (e != hipSuccess) return e;
  *price_per_cu = std::min(std::min(occ[0], occ[1]), std::min(occ[2], occ[3]));
  if (cmode)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(update_per_cu, k_update_c<kUpdateBlock>, kUpdateBlock,
                                                        compact_lds_bytes(ld));
  if (blk == kUpdateBlock)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(update_per_cu, k_update<kUpdateBlock>, kUpdateBlock, lds);
  if (blk > 0)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(update_per_cu, k_update<2 * kUpdateBlock>, 2 * kUpdateBlock,
                                                        lds);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(update_per_cu, k_update_wide<kUpdateBlock>, kUpdateBlock, lds);
}

hipError_t launch_init(const DevLP& lp, const double* b, const double* c, double sense, hipStream_t s) {
  const size_t work = (size_t)lp.m * lp.ld;
  const int grid = (int)std::min<size_t>(4096, (work + 255) / 256 + 1);
  hipLaunchKernelGGL(k_init, dim3(grid), dim3(256), 0, s, lp, b, c, sense);
  return hipGetLastError();
}

hipError_t launch_price(const DevLP& lp, int grid, hipStream_t s) {
  if (lp.a_nt)
    hipLaunchKernelGGL(k_price<true>, dim3(grid), dim3(kPriceBlock), price_lds_bytes(lp.ld), s, lp);
  else
    hipLaunchKernelGGL(k_price<false>, dim3(grid), dim3(kPriceBlock), price_lds_bytes(lp.ld), s, lp);
  return hipGetLastError();
}

hipError_t launch_update(const DevLP& lp, int grid, hipStream_t s) {
  if (lp.cmode)
    hipLaunchKernelGGL(k_update_c<kUpdateBlock>, dim3(grid), dim3(kUpdateBlock), compact_lds_bytes(lp.ld), s, lp);
  else if (lp.upd_block < 0)
    hipLaunchKernelGGL(k_update_wide<kUpdateBlock>, dim3(grid), dim3(kUpdateBlock), wide_lds_bytes(lp.ld), s, lp);
  else if (lp.upd_block == kUpdateBlock)
    hipLaunchKernelGGL(k_update<kUpdateBlock>, dim3(grid), dim3(kUpdateBlock), update_lds_bytes(lp.ld), s, lp);
  else
    hipLaunchKernelGGL(k_update<2 * kUpdateBlock>, dim3(grid), dim3(2 * kUpdateBlock), update_lds_bytes(lp.ld), s,
                       lp);
  return hipGetLastError();
}

hipError_t launch_materialize(const DevLP& lp, hipStream_t s) {
  const size_t work = (size_t)lp.m * lp.ld;
  const int grid = (int)std::max<size_t>(1, std::min<size_t>(4096, (work + 255) / 256));
  hipLaunchKernelGGL(k_materialize, dim3(grid), dim3(256), 0, s, lp);
  return hipGetLastError();
}

hipError_t launch_rebuild_compact(const DevLP& lp, int nd_prev, hipStream_t s) {
  const size_t work = (size_t)lp.m * lp.ld;
  const int grid = (int)std::max<size_t>(1, std::min<size_t>(4096, (work + 255) / 256));
  hipLaunchKernelGGL(k_rebuild_compact, dim3(grid), dim3(256), 0, s, lp, nd_prev);
  return hipGetLastError();
}

hipError_t launch_finish(const DevLP& lp, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, s, lp);
  return hipGetLastError();
}

hipError_t launch_fetch_row(const Ctrl* ctl, const double* host, const double* res, int res_lo, int ld, double* row,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_fetch_row, dim3((ld + 255) / 256), dim3(256), 0, s, ctl, host, res, res_lo, ld, row);
  return hipGetLastError();
}

hipError_t launch_clear_flag(int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, s, flag);
  return hipGetLastError();
}

hipError_t launch_hash(const double* x, size_t nx, uint64_t base, const double* y, size_t ny, const double* z,
                       size_t nz, unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(64), 0, s, out);
  const size_t work = std::max(nx, std::max(ny, nz));
  const int grid = (int)std::max<size_t>(1, std::min<size_t>(2048, (work + 255) / 256));
  hipLaunchKernelGGL(k_hash, dim3(grid), dim3(256), 0, s, x, nx, base, y, ny, z, nz, out);
  return hipGetLastError();
}

hipError_t launch_pack_lp(double* dA, int ld, const double* A, int m, int n, double* b0, const double* b, double* c0,
                          const double* c, int32_t* flag, hipStream_t s) {
  const size_t work = std::max<size_t>((size_t)ld * n, (size_t)std::max(m, n));
  const int grid = (int)std::min<size_t>(4096, (work + 255) / 256);
  hipLaunchKernelGGL(k_pack_lp, dim3(grid), dim3(256), 0, s, dA, ld, A, m, n, b0, b, c0, c, flag);
  return hipGetLastError();
}

hipError_t launch_arm(Ctrl* ctl, int64_t max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_arm, dim3(1), dim3(64), 0, s, ctl, max_iter);
  return hipGetLastError();
}

hipError_t launch_solution(const DevLP& lp, const double* c, double ysign, double* x, double* y, double* objective,
                           hipStream_t s) {
  const int grid = (int)std::min<int>(256, (std::max(lp.m, lp.n) + 255) / 256);
  hipLaunchKernelGGL(k_solution, dim3(grid), dim3(256), 0, s, lp, c, ysign, x, y, objective);
  return hipGetLastError();
}

hipError_t launch_check_finite(const double* x, int64_t count, double bound, int32_t* flag, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(2048, (count + 255) / 256);
  hipLaunchKernelGGL(k_check_finite, dim3(grid), dim3(256), 0, s, x, count, bound, flag);
  return hipGetLastError();
}

}  // namespace lpgpu
