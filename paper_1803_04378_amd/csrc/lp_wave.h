// Wavefront-level building blocks shared by the single-LP kernels and the batched
// solver (gfx950, wave64).  Everything here is deterministic: dot products are a fixed
// per-lane fma chain plus a fixed xor butterfly, and minima are lexicographic on
// (value, index), so no result depends on launch shape or on scheduling.
#pragma once
#include <hip/hip_runtime.h>
#include <limits.h>

namespace lpgpu {
namespace detail {

#ifndef LPGPU_BATCH
#define LPGPU_BATCH 8
#endif
constexpr int kBatch = LPGPU_BATCH;
// Pricing streams A' with the non-temporal hint: A' (8mn bytes) is read once per
// iteration and would otherwise evict B^-1, which k_update reads and rewrites right
// after and which fits in the 256 MB MALL at m = 4000 (measured: k_price 61.8 -> 45.6 us,
// k_update 47.8 -> 43.7 us at 4000 x 8000).
#ifndef LPGPU_STREAM_A
#define LPGPU_STREAM_A 1
#endif
constexpr bool kStreamA = LPGPU_STREAM_A != 0;

__device__ __forceinline__ bool lex_less(double d1, int j1, double d2, int j2) {
  return (d1 < d2) | ((d1 == d2) & (j1 < j2));  // bitwise: no branch
}

// Wavefront reductions without LDS traffic, in DPP lane moves (VALU operand modifiers).
// Inside each row of 16 lanes four moves pair every lane with a partner holding a
// disjoint set of lanes: quad_perm xor 1 (0xB1), quad_perm xor 2 (0x4E), mirror within
// half-rows of 8 (0x141), mirror within the row (0x140); after them every lane holds its
// row's result.  row_bcast:15 (0x142) into rows 1 and 3 and row_bcast:31 (0x143) into
// rows 2 and 3 then gather all four rows in the last row (rows a move does not write
// keep the identity passed as `old`), and lane 63 is read into a wave-uniform value.
// Every combine joins disjoint sets, so operations that are not idempotent (integer
// sums, the two smallest values) are exact too.  Every lane of the wavefront must be
// active.  Used for minima and integer sums only: these do not depend on the order.
template <int CTRL, int RM>
__device__ __forceinline__ int dpp_move(int v, int old) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, RM, 0xF, false);
}
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_move(double v, double old) {
  const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
  const int lo = dpp_move<CTRL, RM>((int)(unsigned)(b & 0xffffffffLL), (int)(unsigned)(o & 0xffffffffLL));
  const int hi = dpp_move<CTRL, RM>((int)(b >> 32), (int)(o >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ int lane63(int v) { return __builtin_amdgcn_readlane(v, 63); }
__device__ __forceinline__ double lane63(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffLL), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// One combine step of each reduction: the partner's value arrives by the DPP move CTRL
// (rows outside RM see the identity).
template <int CTRL, int RM>
__device__ __forceinline__ void lex_step(double& d, int& j) {
  const double d2 = dpp_move<CTRL, RM>(d, __builtin_inf());
  const int j2 = dpp_move<CTRL, RM>(j, INT_MAX);
  const bool take = lex_less(d2, j2, d, j);
  d = take ? d2 : d;
  j = take ? j2 : j;
}
template <int CTRL, int RM>
__device__ __forceinline__ void lex_step_p(double& d, int& j, int& p) {
  const double d2 = dpp_move<CTRL, RM>(d, __builtin_inf());
  const int j2 = dpp_move<CTRL, RM>(j, INT_MAX);
  const int p2 = dpp_move<CTRL, RM>(p, 0);
  const bool take = lex_less(d2, j2, d, j);
  d = take ? d2 : d;
  j = take ? j2 : j;
  p = take ? p2 : p;
}
template <int CTRL, int RM>
__device__ __forceinline__ void two_step(double& t1, double& t2) {
  const double o1 = dpp_move<CTRL, RM>(t1, __builtin_inf()), o2 = dpp_move<CTRL, RM>(t2, __builtin_inf());
  const double n1 = fmin(t1, o1);
  t2 = fmin(fmax(t1, o1), fmin(t2, o2));
  t1 = n1;
}

// Lexicographic minimum of (d, j) over the wavefront, returned in every lane.
__device__ __forceinline__ void wave_lexmin(double& d, int& j) {
  lex_step<0xB1, 0xF>(d, j);
  lex_step<0x4E, 0xF>(d, j);
  lex_step<0x141, 0xF>(d, j);
  lex_step<0x140, 0xF>(d, j);
  lex_step<0x142, 0xA>(d, j);
  lex_step<0x143, 0xC>(d, j);
  d = lane63(d);
  j = lane63(j);
}

// The same carrying a payload p of the winning lane along.
__device__ __forceinline__ void wave_lexmin_payload(double& d, int& j, int& p) {
  lex_step_p<0xB1, 0xF>(d, j, p);
  lex_step_p<0x4E, 0xF>(d, j, p);
  lex_step_p<0x141, 0xF>(d, j, p);
  lex_step_p<0x140, 0xF>(d, j, p);
  lex_step_p<0x142, 0xA>(d, j, p);
  lex_step_p<0x143, 0xC>(d, j, p);
  d = lane63(d);
  j = lane63(j);
  p = lane63(p);
}

// The two smallest values (t1 <= t2) of the wavefront's pairs, in every lane.
__device__ __forceinline__ void wave_two_smallest(double& t1, double& t2) {
  two_step<0xB1, 0xF>(t1, t2);
  two_step<0x4E, 0xF>(t1, t2);
  two_step<0x141, 0xF>(t1, t2);
  two_step<0x140, 0xF>(t1, t2);
  two_step<0x142, 0xA>(t1, t2);
  two_step<0x143, 0xC>(t1, t2);
  t1 = lane63(t1);
  t2 = lane63(t2);
}

__device__ __forceinline__ int wave_min_int(int v) {
  v = min(v, dpp_move<0xB1, 0xF>(v, INT_MAX));
  v = min(v, dpp_move<0x4E, 0xF>(v, INT_MAX));
  v = min(v, dpp_move<0x141, 0xF>(v, INT_MAX));
  v = min(v, dpp_move<0x140, 0xF>(v, INT_MAX));
  v = min(v, dpp_move<0x142, 0xA>(v, INT_MAX));
  v = min(v, dpp_move<0x143, 0xC>(v, INT_MAX));
  return lane63(v);
}
__device__ __forceinline__ int wave_sum_int(int v) {
  v += dpp_move<0xB1, 0xF>(v, 0);
  v += dpp_move<0x4E, 0xF>(v, 0);
  v += dpp_move<0x141, 0xF>(v, 0);
  v += dpp_move<0x140, 0xF>(v, 0);
  v += dpp_move<0x142, 0xA>(v, 0);
  v += dpp_move<0x143, 0xC>(v, 0);
  return lane63(v);
}
__device__ __forceinline__ double wave_min(double v) {
  v = fmin(v, dpp_move<0xB1, 0xF>(v, __builtin_inf()));
  v = fmin(v, dpp_move<0x4E, 0xF>(v, __builtin_inf()));
  v = fmin(v, dpp_move<0x141, 0xF>(v, __builtin_inf()));
  v = fmin(v, dpp_move<0x140, 0xF>(v, __builtin_inf()));
  v = fmin(v, dpp_move<0x142, 0xA>(v, __builtin_inf()));
  v = fmin(v, dpp_move<0x143, 0xC>(v, __builtin_inf()));
  return lane63(v);
}

// Floating-point sum: a fixed xor butterfly (its order is part of every dot product's
// rounding, which the batched solver reproduces).
__device__ __forceinline__ double wave_sum(double a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
  return a;
}

// Block-wide reductions.  Every thread of the block must call them.
template <int BLOCK>
__device__ void block_lexmin(double& d, int& j, double* sd, int* sj) {
  constexpr int W = BLOCK / 64;
  wave_lexmin(d, j);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sd[wave] = d;
    sj[wave] = j;
  }
  __syncthreads();
  d = sd[0];
  j = sj[0];
  for (int w = 1; w < W; ++w)
    if (lex_less(sd[w], sj[w], d, j)) {
      d = sd[w];
      j = sj[w];
    }
  __syncthreads();  // sd, sj may be reused at once
}

template <int BLOCK>
__device__ double block_min(double v, double* sd, int* sj) {
  int dummy = 0;
  block_lexmin<BLOCK>(v, dummy, sd, sj);
  return v;
}

template <int BLOCK>
__device__ int block_min_int(int v, int* si) {
  constexpr int W = BLOCK / 64;
  v = wave_min_int(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) si[wave] = v;
  __syncthreads();
  v = INT_MAX;
  for (int w = 0; w < W; ++w) v = min(v, si[w]);
  __syncthreads();  // si may be reused at once
  return v;
}

template <int BLOCK>
__device__ int block_sum_int(int v, int* si) {
  constexpr int W = BLOCK / 64;
  v = wave_sum_int(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) si[wave] = v;
  __syncthreads();
  v = 0;
  for (int w = 0; w < W; ++w) v += si[w];
  __syncthreads();  // si may be reused at once
  return v;
}

// An integer sum and an integer minimum over the block in one exchange (si holds
// 2 * BLOCK / 64 entries).
template <int BLOCK>
__device__ void block_sum_min_int(int& s, int& mn, int* si) {
  constexpr int W = BLOCK / 64;
  s = wave_sum_int(s);
  mn = wave_min_int(mn);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    si[wave] = s;
    si[W + wave] = mn;
  }
  __syncthreads();
  s = 0;
  mn = INT_MAX;
  for (int w = 0; w < W; ++w) {
    s += si[w];
    mn = min(mn, si[W + w]);
  }
  __syncthreads();  // si may be reused at once
}

// Streaming helpers.  Lane l of a wavefront owns elements l, l+64, l+128, ... of a
// contiguous FP64 vector held as n2 double2; a batch is NB such elements per lane (the
// size of the register array passed in: 16 KB per wavefront in flight at NB = kBatch = 8).
// Every dot product below is the lane's fma chain over its elements in ascending order
// followed by the xor butterfly, whatever the batching, so results depend neither on NB
// nor on launch shape.
typedef double v2d __attribute__((ext_vector_type(2)));

template <int NB>
__device__ __forceinline__ void load_batch(const double2* __restrict__ x, int k0, int n2, double2 (&v)[NB]) {
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int k = k0 + 64 * u;
    if (k < n2) v[u] = x[k];
  }
}

// The same with the non-temporal hint (streamed data that should not displace the
// matrix the next kernel re-reads).
template <int NB>
__device__ __forceinline__ void load_batch_nt(const double2* __restrict__ x, int k0, int n2, double2 (&v)[NB]) {
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int k = k0 + 64 * u;
    if (k < n2) {
      const v2d t = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(x + k));
      v[u] = make_double2(t.x, t.y);
    }
  }
}

// dot(x, y) with x in HBM and y in LDS; `pre` says v already holds the first batch.
template <bool NT, int NB>
__device__ __forceinline__ double wave_dot(const double2* __restrict__ x, const double2* y, int n2, int lane,
                                           double2 (&v)[NB], bool pre) {
  double acc = 0.0;
  for (int k0 = lane; k0 < n2; k0 += 64 * NB) {
    if (!pre) {
      if (NT) load_batch_nt(x, k0, n2, v);
      else load_batch(x, k0, n2, v);
    }
    pre = false;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int k = k0 + 64 * u;
      if (k < n2) {
        const double2 w = y[k];
        acc = fma(v[u].x, w.x, acc);
        acc = fma(v[u].y, w.y, acc);
      }
    }
  }
  return wave_sum(acc);
}

// row <- row + na * rho (in place), returning dot(new row, a) when DOT.  An element pair
// whose rho entries are both zero is unchanged by the fma, so it is not written back
// (the pivot row of B^-1 has a zero wherever the column belongs to a basic slack).
template <bool DOT, int NB>
__device__ __forceinline__ double wave_update_dot(double2* __restrict__ row, const double2* rho, const double2* a,
                                                  double na, int n2, int lane, double2 (&v)[NB], bool pre) {
  double acc = 0.0;
  for (int k0 = lane; k0 < n2; k0 += 64 * NB) {
    if (!pre) load_batch(row, k0, n2, v);
    pre = false;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int k = k0 + 64 * u;
      if (k < n2) {
        const double2 rr = rho[k];
        v[u].x = fma(na, rr.x, v[u].x);
        v[u].y = fma(na, rr.y, v[u].y);
        if (rr.x != 0.0 || rr.y != 0.0) row[k] = v[u];
        if (DOT) {
          const double2 w = a[k];
          acc = fma(v[u].x, w.x, acc);
          acc = fma(v[u].y, w.y, acc);
        }
      }
    }
  }
  return DOT ? wave_sum(acc) : 0.0;
}

// Row r of the new B^-1 is rho itself: write it and (when DOT) dot it with a.
template <bool DOT>
__device__ __forceinline__ double wave_store_dot(double2* __restrict__ row, const double2* rho, const double2* a,
                                                 int n2, int lane) {
  double acc = 0.0;
  for (int k = lane; k < n2; k += 64) {
    const double2 v = rho[k];
    row[k] = v;
    if (DOT) {
      const double2 w = a[k];
      acc = fma(v.x, w.x, acc);
      acc = fma(v.y, w.y, acc);
    }
  }
  return DOT ? wave_sum(acc) : 0.0;
}


}  // namespace detail
}  // namespace lpgpu
