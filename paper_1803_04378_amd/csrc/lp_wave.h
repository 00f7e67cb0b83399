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
  return d1 < d2 || (d1 == d2 && j1 < j2);
}

__device__ __forceinline__ void wave_lexmin(double& d, int& j) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double d2 = __shfl_xor(d, off);
    const int j2 = __shfl_xor(j, off);
    if (lex_less(d2, j2, d, j)) {
      d = d2;
      j = j2;
    }
  }
}

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
  if (wave == 0) {
    d = lane < W ? sd[lane] : __builtin_inf();
    j = lane < W ? sj[lane] : INT_MAX;
    wave_lexmin(d, j);
    if (lane == 0) {
      sd[0] = d;
      sj[0] = j;
    }
  }
  __syncthreads();
  d = sd[0];
  j = sj[0];
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
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) si[wave] = v;
  __syncthreads();
  if (wave == 0) {
    v = lane < W ? si[lane] : INT_MAX;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
    if (lane == 0) si[0] = v;
  }
  __syncthreads();
  return si[0];
}

template <int BLOCK>
__device__ int block_sum_int(int v, int* si) {
  constexpr int W = BLOCK / 64;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) si[wave] = v;
  __syncthreads();
  if (wave == 0) {
    v = lane < W ? si[lane] : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) si[0] = v;
  }
  __syncthreads();
  return si[0];
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
