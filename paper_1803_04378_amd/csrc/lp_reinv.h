// Reinversion of the basis (lp_reinv.hip): B^-1, x_B, W and z recomputed in FP64 from the
// basis list and A', replacing the values the product-form updates have carried.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lp_device.h"

namespace lpgpu {

struct ReinvState;  // grow-only work buffers and the BLAS handle of one LP handle

// Runs one reinversion on stream s.  b is the right-hand side on the device.  Blocks
// until the basis has been read back (the rest is queued on s).  Returns an LP_* code;
// a numerically singular basis block is not an error: the device state is then left as
// it was and Ctrl::n_reinv_failed counts it.
int reinvert(const DevLP& d, const double* b, ReinvState** state, hipStream_t s, int* k_out);
// Creates the work state and the BLAS handle (loading the BLAS kernels once per process)
// and allocates the work memory of small basis blocks for an LP with m rows.
int reinv_prepare(ReinvState** state, int m, int ld);
void reinv_free(ReinvState* state);

}  // namespace lpgpu
