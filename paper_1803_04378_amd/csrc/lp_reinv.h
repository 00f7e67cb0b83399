// Reinversion of the basis (lp_reinv.hip): B^-1, x_B, W and z recomputed in FP64 from the
// basis list and A', replacing the values the product-form updates have carried.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lp_device.h"

namespace lpgpu {

struct ReinvState;  // grow-only work buffers and the BLAS handle of one LP handle

// Queues one reinversion on stream s (nothing waits on the device unless a work buffer
// has to grow).  b is the right-hand side on the device; k is the number of structural
// columns in the basis and nd_old the length of the list D, both from the control block
// as last read back.  Returns an LP_* code; a numerically singular basis block is not an
// error: the device state is then left as it was and Ctrl::n_reinv_failed counts it.
int reinvert(const DevLP& d, const double* b, ReinvState** state, hipStream_t s, int k, int nd_old, int* k_out);
// Creates the work state and the BLAS handle (loading the BLAS kernels once per process),
// allocates the work memory of small basis blocks for an LP with m rows and, once per
// handle, runs the large-block path on a stand-in block so that no first-use cost of the
// BLAS library falls inside a solve.
int reinv_prepare(ReinvState** state, int m, int ld);
void reinv_free(ReinvState* state);

}  // namespace lpgpu
