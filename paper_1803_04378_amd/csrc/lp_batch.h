// Device layout of a batch of LPs for the persistent batched solver (lp_batch.hip).
//
// All LPs live in pooled arrays; BatchLP holds each one's sizes and element offsets.
// Per LP:  A' ld x n column-major (ld = m rounded up to 8), b (m), c (n), B^-1 m x ld
// row-major scratch, gen/excl (2*(n+m) ints), pivot log and tabu list (cap entries
// each), and the final x_B / basis (m each).
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

// LDS bytes one LP needs (rounded to 16).
size_t batch_lds_bytes(int m, int n);
hipError_t launch_batch(const BatchDev& bd, int grid, size_t lds, hipStream_t s);
hipError_t batch_occupancy(int* per_cu, size_t lds);

}  // namespace lpgpu
