// Device-side state of one LP and the kernels of one simplex iteration (gfx950).
//
// Layout in HBM (all FP64 unless stated; ld = m rounded up to a multiple of 8, the
// padding is zero and stays zero):
//   A      ld x n   column-major: column j of A' is contiguous (pricing streams it)
//   Binv   m x ld   row-major:    row i of B^-1 is contiguous (update + FTRAN stream it)
//   W0, W1, rho ld  W = chat_B^T B^-1 (top row of the Figure 1 tableau, two copies: one is
//                   read while the next is written), rho = pivot row / alpha_r
//   dlist, inD      m int32 each: the columns of B^-1 that may differ from unit vectors
//   Bc     m x ld   row-major, rows with ld >= 1024 only: column a holds column dlist[a]
//                   of B^-1 (a < |D|; zero beyond), so that the update and FTRAN read a row's
//                   entries on D contiguously; rho_c (ld) is rho at those columns
//   xB, alpha[2]    m
//   chat            n + m   (minimisation costs; slacks 0)
//   basis (m), pos (n+m), tabu_until (n+m), the leaving-side tabu list, the pivot log: int32
#pragma once
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

namespace lpgpu {

constexpr int kStatusRunning = 0;
constexpr int kStatusOptimal = 1;
constexpr int kStatusUnbounded = 2;
constexpr int kStatusIterLimit = 3;
constexpr int kStatusNumerical = 4;
constexpr int kStatusInfeasible = 5;
// k_update's verdict in the mixed form when the re-priced shortlist holds no improving
// column: no pivot this iteration; the next k_price32 runs the full FP64 pricing pass.
constexpr int kVerdictFallback = 16;

constexpr int kFlagDegenerate = 1;
constexpr int kFlagTie = 2;
constexpr int kFlagAspiration = 4;
constexpr int kFlagLClear = 8;
constexpr int kFlagDriveOut = 16;

// pos[v] of an artificial variable (two-phase start) that has left the basis: any value
// >= 0 keeps a column out of pricing, and this one names no row.
constexpr int kPosBarred = INT_MAX;

#ifndef LPGPU_PRICE_BLOCK
#define LPGPU_PRICE_BLOCK 512
#endif
#ifndef LPGPU_UPDATE_BLOCK
#define LPGPU_UPDATE_BLOCK 512
#endif
constexpr int kPriceBlock = LPGPU_PRICE_BLOCK;
constexpr int kUpdateBlock = LPGPU_UPDATE_BLOCK;
#ifndef LPGPU_FINISH_BLOCK
#define LPGPU_FINISH_BLOCK LPGPU_UPDATE_BLOCK
#endif
constexpr int kFinishBlock = LPGPU_FINISH_BLOCK;  // the one workgroup of k_finish
// Rows of B^-1 one wavefront of k_update may own (the host sizes the grid to respect it).
constexpr int kMaxRowsPerWave = 8;
// Mixed form: FP32 screening keeps this many candidates per workgroup and overall.
constexpr int kShortlist = 16;
constexpr int kPrice32Block = 1024;

// Control block: written by one thread of a kernel (or by the host between solves), read
// by every workgroup of the next kernel; a field is never read and written by different
// workgroups of the same launch.
struct Ctrl {
  int32_t status;
  int32_t q;      // entering variable chosen by the latest pricing, -1 if none
  int32_t r;      // row of the pivot whose B^-1 update is still pending, -1 if none
  int32_t cur;    // alpha[cur] holds the pending pivot's entering column alpha
  int64_t t;      // pivots done
  int64_t max_iter;
  double dq;      // reduced cost d_q of q
  double z;       // objective chat_B^T x_B (minimisation form)
  int32_t ray;    // entering column that proved unboundedness
  int32_t nL;     // entries in the leaving-side tabu list
  int32_t flags;  // pivot-log flags gathered for the pivot in progress
  int32_t pad0;
  int32_t verdict;  // pricing verdict left by k_update for k_finish (-1: k_update did not run)
  int32_t fb;       // mixed form: the next k_price32 runs the full FP64 pricing pass
  int64_t n_degenerate, n_tie, n_aspiration, n_lclear;
  int32_t nsb;   // structural variables in the basis
  int32_t pad1;
  int64_t price_launches;       // pricing passes that ran
  int64_t price_cols;           // structural columns those passes streamed
  int64_t update_launches;      // update passes that ran
  int64_t update_rows_written;  // B^-1 rows those passes rewrote
  double theta;   // step length of the pending pivot
  double pdq;     // reduced cost of the pending pivot's entering variable
  double ar;      // pivot element alpha_r of the pending pivot
  int32_t wcur;   // W0 or W1 holds the top row W of the tableau before the pending pivot
  int32_t pad2;
  int64_t price32_launches;  // mixed form: FP32 screening passes that ran
  int64_t full_prices;       // mixed form: iterations whose shortlist held no improving column
  int64_t n_reinv;           // reinversions installed
  int64_t n_reinv_failed;    // reinversions abandoned on a zero pivot (state kept as it was)
  int64_t rho_nz2;           // element pairs of the pending rho with a nonzero entry
  int64_t update_bytes;      // algorithmic bytes the update passes moved
  int32_t nD;                // columns in the list D (below)
  int32_t pad5;
  int64_t n_fallback;        // mixed form: iterations that ended with kVerdictFallback (no pivot)
  // Taken by k_update for k_price_fin (the ratio-test finish fused with the next pricing
  // pass), whose workgroup 0 rewrites the live fields while the others still read: t, z,
  // the length of D, the structural count, the tabu list's length and the alpha buffer.
  int64_t snap_t;
  double snap_z;
  int32_t snap_nD, snap_nsb, snap_nL, snap_cur;
  // Left by k_price_fin for the next k_update: basis[r] = q_pend (bpend != 0), and the
  // tabu list's generation bump gen[gen_q] = gen_val (gen_q >= 0).
  int32_t q_pend, bpend, gen_q, gen_val;
  // Compact columns (Bc): the index in D the latest finished pivot appended (the leaving
  // slack's column), -1 if none.  Its entry in row r of Bc is not stored yet: it is the
  // unit column's 1.
  int32_t dapp;
  // Left by k_price_fin for the next k_update: inD[ind_pend] = 1 (>= 0), the leaving
  // slack's membership in D, which the finish in every workgroup reads as it was.
  int32_t ind_pend;
};

struct DevLP {
  int32_t m, n, ld;
  int32_t upd_block;  // k_update's workgroup size, update_block(ld), fixed at creation (negative:
                      //   k_update_wide with that many threads)
  const double* A;
  const double* chat;
  double* Binv;
  double* xB;
  double* W0;     // W ping-pong: pricing forms W + d_q rho for the pending pivot from
  double* W1;     //   one copy and one workgroup stores it in the other
  double* rho;
  double* alpha0;
  double* alpha1;
  int32_t* basis;
  // Columns of B^-1 that may differ from a unit vector: every column whose slack has left
  // the basis at some point since the last reinversion (append-only), with a membership
  // flag per column.  A column outside D is e_p for the row p holding its basic slack,
  // exactly: the update never changes it (its rho entry is zero) until that slack leaves.
  int32_t* dlist;
  int32_t* inD;
  int32_t* pos;
  int32_t* tabu_until;
  int32_t* gen;   // generation of each variable's tabu list (bumped to clear it)
  int32_t* excl;  // scratch stamp per variable for list membership tests
  int32_t* Lq;    // list entries: (entering q, leaving variable, generation of q's list)
  int32_t* Ll;
  int32_t* Lgen;
  int32_t* log_enter;
  int32_t* log_row;
  int32_t* log_leave;
  int32_t* log_flags;
  double* part_d;  // pricing partials: 2 per workgroup (all improving, non-tabu improving)
  int32_t* part_j;
  double* part_th;   // update partials per workgroup: min ratio and the lowest row attaining it,
  int32_t* part_low;  // and the two smallest tie thresholds tau of its rows
  double* part_t1;
  double* part_t2;
  double* part_al;    // for the lowest row attaining the min ratio: its alpha, and its basic
  int32_t* part_bv;   //   variable v as 2v + 1 when v is structural or a slack in list D, else 2v
  Ctrl* ctrl;
  int64_t log_cap;
  int32_t price_grid;   // workgroups of k_price (partials to reduce)
  int32_t update_grid;  // workgroups of k_update
  int32_t Lcap;
  int32_t tenure;
  int32_t use_llist;
  int32_t pad1;
  double eps_d, eps_p, eps_z, eps_t;
  // Mixed form only (mixed == 0: the pointers are unused).
  int32_t mixed;
  int32_t sl_k;          // shortlist length K <= kShortlist
  const float* A32;      // FP32 copy of A', same ld x n layout
  uint64_t* part32;      // FP32 screening: kShortlist candidate keys per k_price32 workgroup,
                         //   ascending (key = order-preserving bits of d32, then j)
  double* sl_d;          // the shortlist re-priced in FP64 (kShortlist entries; j = INT_MAX
  int32_t* sl_j;         //   marks an empty slot)
  int32_t price32_grid;  // workgroups of k_price32
  int32_t pad2;
  // Two-phase start only (nullptr otherwise): art[i] = 1 when the unit column n+i is the
  // artificial variable of row i; such a variable is barred (pos = kPosBarred) once it
  // leaves the basis.
  const int8_t* art;
  // Rows of B^-1 that k_update processes: row_lo..row_hi-1, row i at Binv + (i - row_lo) ld
  // (0..m-1 unless the out-of-core panel mode launches it once per panel).
  int32_t row_lo, row_hi;
  // Out-of-core panel mode: device copy of row r of B^-1 for the pricing kernel (nullptr:
  // row r is read from Binv).
  const double* rowsrc;
  // Compact columns (ld >= kSparseMinLd, both precision forms): B^-1 lives in Bc (column a = column
  // dlist[a], zero for a >= |D|; the columns outside D are the unit vectors e_p of the rows
  // p holding their slacks, never stored), rho_c[a] = rho at column dlist[a].  Binv is then
  // brought up to date only on request (k_materialize), for the steps that read B^-1 by
  // its own columns: the tableau read-back, the phase switch, the reinversion.
  int32_t cmode;
  // The pricing kernels read A' with non-temporal loads (it exceeds the last-level cache).
  int32_t a_nt;
  double* Bc;
  double* rho_c;
};

// The top row W this iteration prices with: W + d_q rho of the pending pivot, which the
// first pricing kernel of the iteration stores in the other copy, or the current copy
// when no pivot is pending.
__device__ __forceinline__ const double* pricing_w(const DevLP& lp) {
  const bool other = lp.ctrl->r >= 0;
  return (lp.ctrl->wcur != 0) != other ? lp.W1 : lp.W0;
}

// Sparse-column mode of the update and FTRAN (k_update and the batched solver take the
// same decision, so their arithmetic stays identical): used while at most ld/8 columns of
// B^-1 can differ from unit vectors, and only for rows long enough (ld >= 1024) that
// skipping the unit columns saves more than the index indirection costs.
constexpr int kSparseMinLd = 1024;
// Largest row stride whose whole rho and a_q k_update stages in LDS; longer rows go to
// k_update_wide.
constexpr int kUpdateStageMaxLd = 9792;
__host__ __device__ __forceinline__ bool sparse_columns(int nD, int ld) {
  return ld >= kSparseMinLd && nD * 8 <= ld;
}
// With compact columns the update sums over D in D order at any |D| (k_update_c); the
// batched solver, whose results equal lp_solve's bit for bit, takes the same rule.
__host__ __device__ __forceinline__ bool compact_columns(int ld) { return ld >= kSparseMinLd; }

// One term of the upload check's hash: the SplitMix64 finaliser (Steele, Lea & Flood,
// OOPSLA 2014) of a double's bit pattern mixed with its index; the hash of an array is the
// wrapping sum of its terms, so it does not depend on the order they are added in.
__host__ __device__ __forceinline__ uint64_t hash_word(uint64_t bits, uint64_t index) {
  uint64_t z = bits ^ (index * 0x9E3779B97F4A7C15ull);
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Launchers (lp_kernels.hip).  grid sizes are chosen by the caller.
hipError_t launch_init(const DevLP& lp, const double* b, const double* c, double sense, hipStream_t s);
hipError_t launch_price(const DevLP& lp, int grid, hipStream_t s);
hipError_t launch_update(const DevLP& lp, int grid, hipStream_t s);
// Compact columns: Binv's columns in D from Bc (the others are unit vectors already), and
// Bc from Binv and the list D (zero beyond |D|, given that it was zero beyond nd_prev, the
// length of D before); no pivot may be pending.
hipError_t launch_materialize(const DevLP& lp, hipStream_t s);
hipError_t launch_rebuild_compact(const DevLP& lp, int nd_prev, hipStream_t s);
hipError_t launch_finish(const DevLP& lp, hipStream_t s);
// Sets *flag when some |x_k| exceeds bound (or is NaN).
hipError_t launch_check_finite(const double* x, int64_t count, double bound, int32_t* flag, hipStream_t s);
// Entry point without allocation: *flag = 0; A' packed into ld x n with zero padding, b and
// c copied, bit 1 of *flag for non-finite data, bit 2 for b_i < 0; the pivot limit armed;
// x, y = ysign W and the objective written to device memory.
hipError_t launch_clear_flag(int32_t* flag, hipStream_t s);
// Out-of-core panel mode: row ctl->r of B^-1 into row (from res for rows >= res_lo, else
// from the host copy, read through its device address).
hipError_t launch_fetch_row(const Ctrl* ctl, const double* host, const double* res, int res_lo, int ld, double* row,
                            hipStream_t s);
// *out = the hash of x (nx doubles, indices base..), then of y (ny, indices base + nx ..) and
// z (nz, after y); out is cleared first.
hipError_t launch_hash(const double* x, size_t nx, uint64_t base, const double* y, size_t ny, const double* z,
                       size_t nz, unsigned long long* out, hipStream_t s);
hipError_t launch_pack_lp(double* dA, int ld, const double* A, int m, int n, double* b0, const double* b, double* c0,
                          const double* c, int32_t* flag, hipStream_t s);
hipError_t launch_arm(Ctrl* ctl, int64_t max_iter, hipStream_t s);
hipError_t launch_solution(const DevLP& lp, const double* c, double ysign, double* x, double* y, double* objective,
                           hipStream_t s);
// Kernel entry points for explicit graph construction.
const void* price_kernel(bool nt);
// k_finish fused with the next k_price (iterations after the first of a launch sequence).
const void* price_fin_kernel(bool nt);
// Whether an ld x n A' is read with non-temporal loads by the pricing kernels: when it is
// larger than the device's last-level cache (the 256 MB MALL of MI355X).
constexpr size_t kLastLevelCacheBytes = (size_t)256 << 20;
bool price_nt(int ld, int n);
const void* update_kernel(int ld);
const void* update_kernel_for_block(int block);
// the update kernel an LP launches: k_update_c with compact columns, else by its block
const void* update_kernel_for(const DevLP& lp);
int update_block(int ld);
const void* finish_kernel();
size_t price_lds_bytes(int ld);
size_t update_lds_bytes(int ld);
// LDS of the update kernel update_block(ld) selects (block < 0: k_update_wide).
size_t update_lds_for_block(int block, int ld);
size_t wide_lds_bytes(int ld);
size_t compact_lds_bytes(int ld);
hipError_t kernel_occupancy(int* price_per_cu, int* update_per_cu, int ld, bool cmode);

// Two-phase start (lp_phase.hip): W and z from their definitions for the current costs,
// and the step-0 pivot that replaces the artificial variable basic in row r (no-op for a
// redundant row).  part_t / part_j hold tabrow_grid(lp) entries, drive one int32.
hipError_t launch_reprice(const DevLP& lp, hipStream_t s);
int tabrow_grid(const DevLP& lp);
hipError_t launch_drive_out(const DevLP& lp, int r, double* part_t, int32_t* part_j, int32_t* drive, hipStream_t s);

// Mixed form (lp_mixed.hip).
hipError_t launch_convert32(const double* A, float* A32, size_t count, hipStream_t s);
hipError_t launch_price32(const DevLP& lp, int grid, hipStream_t s);
hipError_t launch_shortlist(const DevLP& lp, hipStream_t s);
const void* price32_kernel();
const void* shortlist_kernel();
size_t price32_lds_bytes(int ld);
int shortlist_block();
hipError_t price32_occupancy(int* per_cu, int ld);
int max_price32_grid();

}  // namespace lpgpu
