// Mixed-precision pricing (gfx950, wave64).
//
// Steps 3-4 of Section 2.1 split into a cheap screening pass and an exact decision:
//   k_price32    FP32 GEMV over an FP32 copy of A' (half the bytes of the FP64 pass):
//                d32_j = chat_j - W32 . a32_j for every nonbasic, non-tabu column, and
//                per workgroup the kShortlist smallest (d32_j, j), ascending.
//   k_shortlist  selects the overall kShortlist smallest of those lists and re-prices
//                the first K of them in FP64, one workgroup per candidate.
// k_update then takes the lexicographic (d, j) minimum among improving shortlisted
// columns.  When none improves, the iteration ends without a pivot (the fallback verdict)
// and the next one prices every column in FP64: k_price32 runs the FP64 pass instead of
// the screening (k_shortlist skips itself), and k_update decides from its partials.
// Optimality and the aspiration case of the tabu rule are therefore always decided in
// FP64.  The re-priced d_j are FP64 dot products like the FP64 pass's, summed in another
// order, so they agree with them to rounding.
#include "lp_device.h"
#include "lp_wave.h"

#include <limits.h>

#include <algorithm>

namespace lpgpu {

using namespace detail;

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// Candidate key: the FP32 reduced cost's bits mapped to an unsigned order (negative values
// bit-inverted, others with the sign bit set) in the high word, the variable index in the
// low word, so that one unsigned compare is the lexicographic (d32, j) order.  NaN never
// becomes a candidate.
__device__ __forceinline__ uint64_t make_key(float d, int j) {
  uint32_t u = __float_as_uint(d);
  u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((uint64_t)u << 32) | (uint32_t)j;
}

__device__ __forceinline__ int key_index(uint64_t key) { return (int)(uint32_t)key; }

constexpr uint64_t kNoKey = ~0ull;

__device__ __forceinline__ float wave_sum32(float a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
  return a;
}

// One batch of x (float4 elements k0, k0 + 64, ...), streamed.
__device__ __forceinline__ void load_batch32(const float4* __restrict__ x, int k0, int n4, float4 (&v)[kBatch]) {
#pragma unroll
  for (int u = 0; u < kBatch; ++u) {
    const int k = k0 + 64 * u;
    if (k < n4) {
      const v4f t = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(x + k));
      v[u] = make_float4(t.x, t.y, t.z, t.w);
    }
  }
}

// FP32 dot(x, y), x streamed from HBM, y in LDS; lane l owns float4 elements l, l+64, ...
// pre: v already holds the first batch.
__device__ __forceinline__ float wave_dot32(const float4* __restrict__ x, const float4* y, int n4, int lane,
                                            float4 (&v)[kBatch], bool pre) {
  float acc = 0.f;
  for (int k0 = lane; k0 < n4; k0 += 64 * kBatch) {
    if (!pre) load_batch32(x, k0, n4, v);
    pre = false;
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int k = k0 + 64 * u;
      if (k < n4) {
        const float4 w = y[k];
        acc = fmaf(v[u].x, w.x, acc);
        acc = fmaf(v[u].y, w.y, acc);
        acc = fmaf(v[u].z, w.z, acc);
        acc = fmaf(v[u].w, w.w, acc);
      }
    }
  }
  return wave_sum32(acc);
}

}  // namespace

__global__ void k_convert32(const double* __restrict__ A, float* __restrict__ A32, size_t count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < count; k += stride) A32[k] = (float)A[k];
}

// Entries of a sorted list of kShortlist (= 16) keys below key: a fixed five-read search.
__device__ __forceinline__ int count_below(const uint64_t* list, uint64_t key) {
  int pos = 0;
  pos += list[pos + 7] < key ? 8 : 0;
  pos += list[pos + 3] < key ? 4 : 0;
  pos += list[pos + 1] < key ? 2 : 0;
  pos += list[pos] < key ? 1 : 0;
  pos += list[pos] < key ? 1 : 0;  // only when pos == 15 can this add
  return pos;
}
// The same for entries at most key.
__device__ __forceinline__ int count_le(const uint64_t* list, uint64_t key) {
  int pos = 0;
  pos += list[pos + 7] <= key ? 8 : 0;
  pos += list[pos + 3] <= key ? 4 : 0;
  pos += list[pos + 1] <= key ? 2 : 0;
  pos += list[pos] <= key ? 1 : 0;
  pos += list[pos] <= key ? 1 : 0;
  return pos;
}
static_assert(kShortlist == 16, "count_below and count_le are written for lists of 16");

// ---------------------------------------------------------------------------------------
// The full FP64 pass of Steps 3-4 (k_price's reduced costs and per-workgroup minima over
// all improving and non-tabu improving columns), run by k_price32's grid in the
// iteration after a fallback verdict.  No pivot is pending then, so the current W is
// the top row; it is read from memory (each d_j is the same wave_dot as k_price's).
__device__ void fp64_pass(const DevLP& lp) {
  constexpr int waves = kPrice32Block / 64;
  __shared__ double red_d[2 * waves];
  __shared__ int red_j[2 * waves];
  const int m = lp.m, n = lp.n, ld2 = lp.ld / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gw = blockIdx.x * waves + wave, nw = gridDim.x * waves;
  const int64_t t = lp.ctrl->t;
  const double* W = lp.ctrl->wcur ? lp.W1 : lp.W0;
  const double2* W2 = reinterpret_cast<const double2*>(W);
  const double neg_eps = -lp.eps_d;
  double da = __builtin_inf(), df = __builtin_inf();
  int ja = INT_MAX, jf = INT_MAX;
  double2 v[kBatch];
  for (int j = gw; j < n; j += nw) {
    if (lp.pos[j] >= 0) continue;
    const double s =
        wave_dot<kStreamA>(reinterpret_cast<const double2*>(lp.A + (size_t)j * lp.ld), W2, ld2, lane, v, false);
    const double d = lp.chat[j] - s;
    if (d < neg_eps) {
      if (lex_less(d, j, da, ja)) {
        da = d;
        ja = j;
      }
      if (lp.tabu_until[j] < t && lex_less(d, j, df, jf)) {
        df = d;
        jf = j;
      }
    }
  }
  for (int i = blockIdx.x * kPrice32Block + threadIdx.x; i < m; i += gridDim.x * kPrice32Block) {
    const int vv = n + i;
    if (lp.pos[vv] >= 0) continue;
    const double d = lp.chat[vv] - W[i];  // a_{n+i} = e_i
    if (d < neg_eps) {
      if (lex_less(d, vv, da, ja)) {
        da = d;
        ja = vv;
      }
      if (lp.tabu_until[vv] < t && lex_less(d, vv, df, jf)) {
        df = d;
        jf = vv;
      }
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

// ---------------------------------------------------------------------------------------
// FP32 screening.  Wave gw prices columns gw, gw + nw, ... of all N = n + m variables
// (slack j = n + i needs no GEMV: d_j = chat_j - W_i).  Each wave keeps its kShortlist
// smallest keys in lanes 0..15, sorted; the workgroup merges its waves' lists by rank.
// Unused slots are written as (+inf, N + slot), distinct per slot, so every key in the
// candidate lists is unique.
__global__ __launch_bounds__(kPrice32Block) void k_price32(DevLP lp) {
  if (lp.ctrl->status != kStatusRunning) return;
  if (lp.ctrl->fb) {
    fp64_pass(lp);
    return;
  }
  constexpr int waves = kPrice32Block / 64;
  constexpr int S = kShortlist;
  extern __shared__ float4 s_w4[];
  __shared__ uint64_t s_key[waves * S];
  const int64_t t = lp.ctrl->t;
  const int r = lp.ctrl->r;
  const int wc = lp.ctrl->wcur;
  const int n = lp.n, N = lp.n + lp.m, n4 = lp.ld / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gw = blockIdx.x * waves + wave;
  const int nw = gridDim.x * waves;

  // Requested before the top row is formed (as in k_price): the state of this wave's
  // columns (lane c holds column gw + c nw).  (Holding a first batch of A' across the
  // staging would cost more registers than this kernel's occupancy allows.)
  const int jl = gw + lane * nw;
  int c_pos = 0, c_tabu = 0;
  double c_chat = 0.0;
  if (jl < N) {
    c_pos = lp.pos[jl];
    c_tabu = lp.tabu_until[jl];
    c_chat = lp.chat[jl];
  }

  // Step 8 on the top row for the pending pivot, as in k_price: W_new = W + d_q rho is
  // formed in FP64 and staged rounded to FP32; workgroup 0 stores rho and W_new.
  float* s_w = reinterpret_cast<float*>(s_w4);
  if (r >= 0 && lp.cmode) {
    // Compact columns (as in k_price): rho is zero outside D and row r of Bc holds it on D
    // (at the index the pivot appended, the unit column's 1, not stored yet); W_new equals
    // W elsewhere.  Workgroup 0 stores W_new (a copy of W, then the entries on D) and rho_c.
    const double* Wold = wc ? lp.W1 : lp.W0;
    double* Wnew = wc ? lp.W0 : lp.W1;
    const double ar = lp.ctrl->ar;
    const double dq = lp.ctrl->pdq;
    const int nDn = lp.ctrl->nD, a_app = lp.ctrl->dapp;
    const double* crow = lp.Bc + (size_t)r * lp.ld;
    const bool writer = blockIdx.x == 0;
    {
      // every load of a round before its stores (a load-store loop waits for each load)
      const double2* Wo2 = reinterpret_cast<const double2*>(Wold);
      double2* Wn2 = reinterpret_cast<double2*>(Wnew);
      const int ld2 = lp.ld / 2;
      constexpr int U = 4;
      for (int k0 = threadIdx.x; k0 < ld2; k0 += U * kPrice32Block) {
        double2 tw[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = k0 + u * kPrice32Block;
          if (k < ld2) tw[u] = Wo2[k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = k0 + u * kPrice32Block;
          if (k < ld2) {
            s_w[2 * k] = (float)tw[u].x;
            s_w[2 * k + 1] = (float)tw[u].y;
            if (writer) Wn2[k] = tw[u];
          }
        }
      }
    }
    __syncthreads();  // (the copy of W is stored before the entries on D overwrite it)
    for (int a = threadIdx.x; a < nDn; a += kPrice32Block) {
      const int j = lp.dlist[a];
      const double rr = (a == a_app ? 1.0 : crow[a]) / ar;
      const double wn = fma(dq, rr, Wold[j]);
      s_w[j] = (float)wn;
      if (writer) {
        Wnew[j] = wn;
        lp.rho_c[a] = rr;
      }
    }
  } else if (r >= 0) {
    const double2* Wold = reinterpret_cast<const double2*>(wc ? lp.W1 : lp.W0);
    double2* Wnew = reinterpret_cast<double2*>(wc ? lp.W0 : lp.W1);
    const double ar = lp.ctrl->ar;
    const double dq = lp.ctrl->pdq;
    const double2* rowr = reinterpret_cast<const double2*>(lp.Binv + (size_t)r * lp.ld);
    double2* rho2 = reinterpret_cast<double2*>(lp.rho);
    const bool writer = blockIdx.x == 0;
    int nz2 = 0;
    for (int k = threadIdx.x; k < lp.ld / 2; k += kPrice32Block) {
      const double2 b = rowr[k];
      const double2 w = Wold[k];
      const double2 rr = make_double2(b.x / ar, b.y / ar);
      const double2 wn = make_double2(fma(dq, rr.x, w.x), fma(dq, rr.y, w.y));
      s_w[2 * k] = (float)wn.x;
      s_w[2 * k + 1] = (float)wn.y;
      if (writer) {
        rho2[k] = rr;
        Wnew[k] = wn;
        nz2 += (rr.x != 0.0 || rr.y != 0.0) ? 1 : 0;
      }
    }
    if (writer) {
      // pairs of rho with a nonzero entry (the update writes only those)
      __shared__ int s_nz[kPrice32Block / 64];
      nz2 = block_sum_int<kPrice32Block>(nz2, s_nz);
      if (threadIdx.x == 0) lp.ctrl->rho_nz2 = nz2;
    }
  } else {
    const double* W = wc ? lp.W1 : lp.W0;
    const double2* W2 = reinterpret_cast<const double2*>(W);
    const int ld2 = lp.ld / 2;
    constexpr int U = 4;
    for (int k0 = threadIdx.x; k0 < ld2; k0 += U * kPrice32Block) {
      double2 tw[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * kPrice32Block;
        if (k < ld2) tw[u] = W2[k];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * kPrice32Block;
        if (k < ld2) {
          s_w[2 * k] = (float)tw[u].x;
          s_w[2 * k + 1] = (float)tw[u].y;
        }
      }
    }
  }
  __syncthreads();

  uint64_t key = kNoKey;  // lane l < S: the wave's l-th smallest key
  uint64_t worst = kNoKey;
  int c = 0;
  for (int j = gw; j < N; j += nw, ++c) {
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
    if (pos >= 0 || tabu >= t) continue;
    float d;
    if (j < n) {
      float4 v[kBatch];
      const float s = wave_dot32(reinterpret_cast<const float4*>(lp.A32 + (size_t)j * lp.ld), s_w4, n4, lane, v, false);
      d = (float)ch - s;
    } else {
      d = (float)ch - s_w[j - n];
    }
    if (d != d) continue;
    const uint64_t kn = make_key(d, j);
    if (kn >= worst) continue;
    // Insert at its rank among lanes 0..S-1; the lanes after it shift up by one.
    const int at = __popcll(__ballot(lane < S && key < kn));
    const uint64_t up = __shfl_up(key, 1);
    if (lane == at) key = kn;
    else if (lane > at && lane < S) key = up;
    worst = __shfl(key, S - 1);
  }
  if (lane < S) s_key[wave * S + lane] = key;
  __syncthreads();
  if (threadIdx.x < waves * S) {
    const int w = threadIdx.x / S, l = threadIdx.x % S;
    const uint64_t k0 = s_key[threadIdx.x];
    // Rank in the union: own position plus, per other wave, the entries before it; equal
    // keys (empty slots) are ordered by wave.  The searches are independent: unrolled and
    // without branches, their LDS reads interleave.
    int rank = l;
#pragma unroll
    for (int w2 = 0; w2 < waves; ++w2) {
      const uint64_t* l2 = s_key + w2 * S;
      const int cb = w2 < w ? count_le(l2, k0) : count_below(l2, k0);
      rank += w2 != w ? cb : 0;
    }
    if (rank < S) {
      const int slot = blockIdx.x * S + rank;
      lp.part32[slot] = k0 != kNoKey ? k0 : make_key(__builtin_inff(), N + slot);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Overall shortlist and its FP64 re-price (every workgroup selects, workgroup w re-prices
// candidate w).  The kShortlist smallest keys of all lists lie in the kShortlist lists
// with the smallest heads: if T is the kShortlist-th smallest head, those heads are
// kShortlist keys <= T, so every key of the overall shortlist is <= T, and any list
// whose head exceeds T holds only larger keys.  All lists are loaded into LDS at once;
// each wavefront sorts 64 heads with a bitonic network in registers, the waves' 16
// smallest heads are ranked by binary search to pick the lists, and the entries of those
// lists are ranked the same way (keys are unique, so ranks are distinct).
constexpr int kShortlistBlock = 512;
constexpr int kMaxLists = kShortlistBlock;


// Elements of a W-length vector one thread of k_shortlist holds (ld / 2 double2 over the
// block, ld <= LP_MAX_ROWS = 9792).
constexpr int kShortlistPer = (9792 / 2 + kShortlistBlock - 1) / kShortlistBlock;

__global__ __launch_bounds__(kShortlistBlock) void k_shortlist(DevLP lp) {
  // The control fields, W and the candidate lists are loaded up front so that their
  // latencies overlap; only the entering column waits for the selection.
  const Ctrl* ctl = lp.ctrl;
  const int status = ctl->status, r = ctl->r, wc = ctl->wcur, fb = ctl->fb;
  if (status != kStatusRunning || fb) return;  // (fb: this iteration runs the FP64 pass)
  constexpr int S = kShortlist;
  constexpr int W = kShortlistBlock / 64;
  __shared__ uint64_t s_all[kMaxLists * S];
  __shared__ uint64_t s_wh[W * S];
  __shared__ int s_wg[W * S];
  __shared__ int s_sel[S];
  __shared__ int s_top[S];
  __shared__ double s_red[W];
  const int G = lp.price32_grid, N = lp.n + lp.m, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int ld2 = lp.ld / 2;
  const double* Wc = (wc != 0) != (r >= 0) ? lp.W1 : lp.W0;  // pricing_w, from the loads above
  double2 wv[kShortlistPer];
#pragma unroll
  for (int u = 0; u < kShortlistPer; ++u) {
    const int k = tid + u * kShortlistBlock;
    wv[u] = k < ld2 ? reinterpret_cast<const double2*>(Wc)[k] : make_double2(0.0, 0.0);
  }
  {
    // every load first, then the stores (a loop of load-then-store waits for each load)
    constexpr int kPer = kMaxLists * S / kShortlistBlock;
    uint64_t kv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * kShortlistBlock;
      kv[u] = e < G * S ? lp.part32[e] : kNoKey;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * kShortlistBlock;
      if (e < G * S) s_all[e] = kv[u];
    }
  }
  if (tid < S) s_sel[tid] = -1;
  __syncthreads();
  // Bitonic sort of this wave's 64 heads (ascending), each carrying its list index.
  const int g0 = wave * 64 + lane;
  uint64_t key = g0 < G ? s_all[g0 * S] : kNoKey;
  int g = g0;
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint64_t ok = __shfl_xor(key, j);
      const int og = __shfl_xor(g, j);
      const bool up = (lane & k) == 0;
      const bool low = (lane & j) == 0;
      const bool take_other = (low == up) ? (ok < key) : (ok > key);
      if (take_other) {
        key = ok;
        g = og;
      }
    }
  }
  if (lane < S) {
    s_wh[wave * S + lane] = key;
    s_wg[wave * S + lane] = g;
  }
  __syncthreads();
  // The searches of one key in the other lists are independent: unrolled and without
  // branches, their LDS reads interleave (six dependent rounds instead of six per list).
  if (tid < W * S) {
    const uint64_t k0 = s_wh[tid];
    int rank = tid % S;
#pragma unroll
    for (int w2 = 0; w2 < W; ++w2) {
      const int cb = count_below(s_wh + w2 * S, k0);
      rank += w2 != tid / S ? cb : 0;
    }
    if (rank < S && k0 != kNoKey) s_sel[rank] = s_wg[tid];
  }
  __syncthreads();
  if (tid < S * S) {
    const int l = tid / S, idx = tid % S;
    const int gl = s_sel[l];
    if (gl >= 0) {
      const uint64_t k0 = s_all[gl * S + idx];
      int rank = idx;
#pragma unroll
      for (int l2 = 0; l2 < S; ++l2) {
        const int sl = s_sel[l2];
        const int cb = count_below(s_all + (sl >= 0 ? sl : 0) * S, k0);
        rank += (l2 != l && sl >= 0) ? cb : 0;
      }
      if (rank < S) s_top[rank] = key_index(k0);
    }
  }
  // The selected lists hold at least S keys (one list has S), so every s_top slot is set.
  __syncthreads();
  // FP64 re-price of candidate w with the whole workgroup: thread t sums elements
  // t, t + 512, ... in an fma chain, then a fixed-order reduction.
  const int w = blockIdx.x;
  const int j = s_top[w];
  const double chat_j = j < N ? lp.chat[j] : 0.0;
  const double w_slack = (j >= lp.n && j < N) ? Wc[j - lp.n] : 0.0;
  double acc = 0.0;
  if (j < lp.n) {
    const double2* a2 = reinterpret_cast<const double2*>(lp.A + (size_t)j * lp.ld);
    double2 av[kShortlistPer];
#pragma unroll
    for (int u = 0; u < kShortlistPer; ++u) {
      const int k = tid + u * kShortlistBlock;
      av[u] = k < ld2 ? a2[k] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kShortlistPer; ++u) {
      acc = fma(av[u].x, wv[u].x, acc);
      acc = fma(av[u].y, wv[u].y, acc);
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) s_red[wave] = acc;
  __syncthreads();
  if (tid == 0) {
    double sdot = 0.0;
    for (int k = 0; k < W; ++k) sdot += s_red[k];
    double d = __builtin_inf();
    int jj = INT_MAX;
    if (j < N) {
      jj = j;
      d = j < lp.n ? chat_j - sdot : chat_j - w_slack;
    }
    lp.sl_d[w] = d;
    lp.sl_j[w] = jj;
  }
}

hipError_t launch_convert32(const double* A, float* A32, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const int grid = (int)std::min<size_t>(8192, (count + 255) / 256);
  hipLaunchKernelGGL(k_convert32, dim3(grid), dim3(256), 0, s, A, A32, count);
  return hipGetLastError();
}

size_t price32_lds_bytes(int ld) { return sizeof(float) * (size_t)ld; }

int shortlist_block() { return kShortlistBlock; }

int max_price32_grid() { return kMaxLists; }

hipError_t launch_price32(const DevLP& lp, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_price32, dim3(grid), dim3(kPrice32Block), price32_lds_bytes(lp.ld), s, lp);
  return hipGetLastError();
}

hipError_t launch_shortlist(const DevLP& lp, hipStream_t s) {
  hipLaunchKernelGGL(k_shortlist, dim3(lp.sl_k), dim3(kShortlistBlock), 0, s, lp);
  return hipGetLastError();
}

const void* price32_kernel() { return reinterpret_cast<const void*>(&k_price32); }
const void* shortlist_kernel() { return reinterpret_cast<const void*>(&k_shortlist); }

hipError_t price32_occupancy(int* per_cu, int ld) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_price32, kPrice32Block, price32_lds_bytes(ld));
}

}  // namespace lpgpu
