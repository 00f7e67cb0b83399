// Device layout of a batch of LPs for the persistent batched solver (lp_batch.hip).
//
// All LPs live in pooled arrays; BatchLP holds each one's sizes and element offsets.
// Per LP:  A' ld x n column-major (ld = m rounded up to 8), b (m), c (n), B^-1 m x ld
// row-major scratch (unused when the LP keeps B^-1 in LDS), gen/excl (2*(n+m) ints),
// pivot log and tabu list (cap entries each), and the final x_B / basis (m each).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpgpu {

constexpr int kBatchBlock = 256;
constexpr int kBatchWaves = kBatchBlock / 64;

struct BatchLP {
  int32_t m, n, ld, waves;  // waves: 1 (one wavefront per LP) or kBatchWaves (whole workgroup)
  int64_t offA, offb, offc, offB, offI, offLog, offOut;
  int64_t cap;              // pivot limit = capacity of its pivot log and tabu list
  int32_t binv_lds;         // 1: B^-1 lives in LDS after the LP's vectors (k_batch<true>)
  int32_t pad;
};

struct BatchDev {
  const BatchLP* lps;
  const int4* items;  // work items: one wide LP in .x, or up to 4 narrow LPs (-1 = none)
  int32_t n_items;
  int32_t slot_bytes;  // LDS bytes of one wavefront's slot in narrow items
  int32_t* queue;      // next work item (atomic counter, zeroed before each launch)
  const double* A;
  const double* b;
  const double* c;
  double* Binv;
  int32_t* iscr;  // gen and excl
  int32_t* log_enter;
  int32_t* log_row;
  int32_t* log_leave;
  int32_t* log_flags;
  int32_t* Lq;
  int32_t* Ll;
  int32_t* Lgen;
  double* xB_out;
  int32_t* basis_out;
  int32_t* status_out;
  int64_t* iters_out;
  double* z_out;
  int32_t* ray_out;
  double sense;
  int32_t tenure;
  int32_t use_llist;
  double eps_d, eps_p, eps_z, eps_t;
};

// LDS one LP needs: W, rho, a_q (ld each), alpha x2, x_B and the ratios (m each) in FP64,
// then basis and the list D with its flags (3m), pos and the tabu marks (2(n+m)) in
// int32, rounded to 16 bytes.  With B^-1 in LDS, its m x ld FP64 follow.
__host__ __device__ inline size_t batch_lds_bytes(int m, int n) {
  const size_t ld = (size_t)(m + 7) / 8 * 8;
  const size_t bytes = 8 * (3 * ld + 4 * (size_t)m) + 4 * (3 * (size_t)m + 2 * ((size_t)n + m));
  return (bytes + 15) / 16 * 16;
}
__host__ __device__ inline size_t batch_lds_bytes_binv(int m, int n) {
  return batch_lds_bytes(m, n) + 8 * (size_t)m * ((size_t)(m + 7) / 8 * 8);
}
// Launches k_batch<binv_lds>: B^-1 in the pooled HBM array, or in LDS.
hipError_t launch_batch(const BatchDev& bd, int grid, size_t lds, bool binv_lds, hipStream_t s);
// The dense law of lp_batch_create_dense into the pools: LP i (layout lps[i], per-LP seed
// h(seed, 7, i)) gets A'_rj ~ U(0,1) at index j m + r, b_r ~ U(1,10), c_j ~ U(1,10), and zero
// padding rows; one workgroup per LP.
hipError_t launch_gen_batch(const BatchLP* lps, int32_t count, uint64_t seed, double* A, double* b, double* c,
                            hipStream_t s);
hipError_t batch_occupancy(int* per_cu, size_t lds, bool binv_lds);

}  // namespace lpgpu
