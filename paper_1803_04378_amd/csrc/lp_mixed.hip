// Mixed-precision pricing (gfx950, wave64).
//
// Steps 3-4 of Section 2.1 split into a cheap screening pass and an exact decision:
//   k_price32    FP32 GEMV over an FP32 copy of A' (half the bytes of the FP64 pass):
//                d32_j = chat_j - W32 . a32_j for every nonbasic, non-tabu column, and
//                per workgroup the kShortlist smallest (d32_j, j), ascending.
//   k_shortlist  merges those lists into the overall kShortlist smallest and re-prices
//                the first K of them in FP64, one workgroup per candidate, with the same
//                per-lane fma chain and butterfly as k_price, so each re-priced d_j is
//                bit-identical to the value the FP64 pass would give that column.
// k_update then takes the lexicographic (d, j) minimum among improving shortlisted
// columns.  When none improves, the FP64 pass k_price (which skips itself otherwise)
// has priced every column, and the decision falls back to it: optimality and the
// aspiration case of the tabu rule are therefore always decided in FP64.
#include "lp_device.h"
#include "lp_wave.h"

#include <limits.h>

#include <algorithm>

namespace lpgpu {

using namespace detail;

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bool key_less(float d1, int j1, float d2, int j2) {
  return d1 < d2 || (d1 == d2 && j1 < j2);
}

__device__ __forceinline__ float wave_sum32(float a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
  return a;
}

// FP32 dot(x, y), x streamed from HBM, y in LDS; lane l owns float4 elements l, l+64, ...
__device__ __forceinline__ float wave_dot32(const float4* __restrict__ x, const float4* y, int n4, int lane) {
  float acc = 0.f;
  for (int k0 = lane; k0 < n4; k0 += 64 * kBatch) {
    float4 v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int k = k0 + 64 * u;
      if (k < n4) {
        const v4f t = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(x + k));
        v[u] = make_float4(t.x, t.y, t.z, t.w);
      }
    }
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

// ---------------------------------------------------------------------------------------
// FP32 screening.  Wave gw prices columns gw, gw + nw, ... of all N = n + m variables
// (slack j = n + i needs no GEMV: d_j = chat_j - W_i, computed in FP64 and rounded).
// Each wave keeps its kShortlist best in lanes 0..15, sorted; the workgroup merges its
// waves' lists by rank.  Unused slots hold (+inf, j >= N), with distinct j per slot, so
// every key in the candidate lists is unique.
__global__ __launch_bounds__(kPrice32Block) void k_price32(DevLP lp) {
  if (lp.ctrl->status != kStatusRunning) return;
  constexpr int waves = kPrice32Block / 64;
  constexpr int S = kShortlist;
  extern __shared__ float4 s_w4[];
  __shared__ float s_cd[waves * S];
  __shared__ int s_cj[waves * S];
  const int64_t t = lp.ctrl->t;
  const int n = lp.n, N = lp.n + lp.m, n4 = lp.ld / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gw = blockIdx.x * waves + wave;
  const int nw = gridDim.x * waves;

  for (int k = threadIdx.x; k < lp.ld; k += kPrice32Block) reinterpret_cast<float*>(s_w4)[k] = (float)lp.W[k];
  __syncthreads();

  float kd = __builtin_inff();
  int kj = INT_MAX;
  float worst_d = __builtin_inff();
  int worst_j = INT_MAX;
  for (int j = gw; j < N; j += nw) {
    if (lp.pos[j] >= 0 || lp.tabu_until[j] >= t) continue;
    float d;
    if (j < n) {
      const float s = wave_dot32(reinterpret_cast<const float4*>(lp.A32 + (size_t)j * lp.ld), s_w4, n4, lane);
      d = (float)lp.chat[j] - s;
    } else {
      d = (float)(lp.chat[j] - lp.W[j - n]);
    }
    if (!key_less(d, j, worst_d, worst_j)) continue;
    // Insert (d, j) at its rank among lanes 0..S-1; the lanes after it shift up by one.
    const bool before = lane < S && key_less(kd, kj, d, j);
    const int at = __popcll(__ballot(before));
    const float ud = __shfl_up(kd, 1);
    const int uj = __shfl_up(kj, 1);
    if (lane == at) {
      kd = d;
      kj = j;
    } else if (lane > at && lane < S) {
      kd = ud;
      kj = uj;
    }
    worst_d = __shfl(kd, S - 1);
    worst_j = __shfl(kj, S - 1);
  }
  if (lane < S) {
    s_cd[wave * S + lane] = kd;
    s_cj[wave * S + lane] = kj;
  }
  __syncthreads();
  if (threadIdx.x < waves * S) {
    const int w = threadIdx.x / S, l = threadIdx.x % S;
    const float d = s_cd[threadIdx.x];
    const int j = s_cj[threadIdx.x];
    // Rank in the union: own position plus, per other wave, the entries before it; equal
    // keys (empty slots) are ordered by wave.
    int rank = l;
    for (int w2 = 0; w2 < waves; ++w2) {
      if (w2 == w) continue;
      int lo = 0, hi = S;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const float d2 = s_cd[w2 * S + mid];
        const int j2 = s_cj[w2 * S + mid];
        const bool prec = key_less(d2, j2, d, j) || (d2 == d && j2 == j && w2 < w);
        if (prec) lo = mid + 1;
        else hi = mid;
      }
      rank += lo;
    }
    if (rank < S) {
      const int slot = blockIdx.x * S + rank;
      lp.part32_d[slot] = d;
      lp.part32_j[slot] = j < N ? j : N + slot;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Merge of the k_price32 lists (every workgroup, redundantly) and the FP64 re-price of
// candidate blockIdx.x.  The lists are merged pairwise in LDS: an entry's rank in the
// merged pair is its position plus the number of entries of the other list below it
// (keys are unique), and only ranks below kShortlist are kept.
constexpr int kShortlistBlock = 1024;
constexpr int kMergeTasks = 8;  // merge tasks per thread at the widest level (512 lists)
constexpr int kMaxLists = kShortlistBlock * kMergeTasks / kShortlist;

__global__ __launch_bounds__(kShortlistBlock) void k_shortlist(DevLP lp) {
  if (lp.ctrl->status != kStatusRunning) return;
  constexpr int S = kShortlist;
  extern __shared__ float s_md[];
  const int G = lp.price32_grid;
  int L = 1;
  while (L < G) L <<= 1;
  int* s_mj = reinterpret_cast<int*>(s_md + L * S);
  const int N = lp.n + lp.m;
  const int tid = threadIdx.x;
  for (int k = tid; k < L * S; k += kShortlistBlock) {
    if (k < G * S) {
      s_md[k] = lp.part32_d[k];
      s_mj[k] = lp.part32_j[k];
    } else {
      s_md[k] = __builtin_inff();
      s_mj[k] = N + k;
    }
  }
  __syncthreads();
  for (int len = L; len > 1; len >>= 1) {
    const int tasks = (len >> 1) * 2 * S;
    float od[kMergeTasks];
    int oj[kMergeTasks], oat[kMergeTasks];
#pragma unroll
    for (int u = 0; u < kMergeTasks; ++u) {
      oat[u] = -1;
      const int e = tid + u * kShortlistBlock;
      if (e < tasks) {
        const int p = e / (2 * S), side = (e / S) & 1, idx = e % S;
        const int mine = (2 * p + side) * S, other = (2 * p + 1 - side) * S;
        const float d = s_md[mine + idx];
        const int j = s_mj[mine + idx];
        int lo = 0, hi = S;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (key_less(s_md[other + mid], s_mj[other + mid], d, j)) lo = mid + 1;
          else hi = mid;
        }
        const int rank = idx + lo;
        if (rank < S) {
          od[u] = d;
          oj[u] = j;
          oat[u] = p * S + rank;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMergeTasks; ++u)
      if (oat[u] >= 0) {
        s_md[oat[u]] = od[u];
        s_mj[oat[u]] = oj[u];
      }
    __syncthreads();
  }
  // FP64 re-price of candidate w by wave 0 (identical arithmetic to k_price).
  const int w = blockIdx.x;
  if (tid >= 64) return;
  const int lane = tid;
  const int j = s_mj[w];
  double d = __builtin_inf();
  int jj = INT_MAX;
  if (j < N) {
    jj = j;
    if (j < lp.n) {
      double2 v[kBatch];
      const double s = wave_dot<false>(reinterpret_cast<const double2*>(lp.A + (size_t)j * lp.ld),
                                       reinterpret_cast<const double2*>(lp.W), lp.ld / 2, lane, v, false);
      d = lp.chat[j] - s;
    } else {
      d = lp.chat[j] - lp.W[j - lp.n];
    }
  }
  if (lane == 0) {
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

size_t shortlist_lds_bytes(int grid32) {
  int L = 1;
  while (L < grid32) L <<= 1;
  return (sizeof(float) + sizeof(int)) * (size_t)L * kShortlist;
}

int max_price32_grid() { return kMaxLists; }

hipError_t launch_price32(const DevLP& lp, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_price32, dim3(grid), dim3(kPrice32Block), price32_lds_bytes(lp.ld), s, lp);
  return hipGetLastError();
}

hipError_t launch_shortlist(const DevLP& lp, hipStream_t s) {
  hipLaunchKernelGGL(k_shortlist, dim3(lp.sl_k), dim3(kShortlistBlock), shortlist_lds_bytes(lp.price32_grid), s,
                     lp);
  return hipGetLastError();
}

const void* price32_kernel() { return reinterpret_cast<const void*>(&k_price32); }
const void* shortlist_kernel() { return reinterpret_cast<const void*>(&k_shortlist); }

hipError_t price32_occupancy(int* per_cu, int ld) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_price32, kPrice32Block, price32_lds_bytes(ld));
}

}  // namespace lpgpu
