// Host-side interface of the adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace stn {

// One reverse step of the leapfrog with c(x): lam2 <- 2 lam1 - lam2 + L8(c lam1)
// (lam1 = lambda_{n+1}, lam2 = lambda_{n+2} on entry and lambda_n on return)
// and g += lam1 * L8(us) in FP64 (us = u_n).  w: the five L8 weights.
hipError_t launch_adjoint_step(bool coef_bf16, const float* lam1, float* lam2, const void* coef,
                               const float* us, double* g, const dims& d, const double* w,
                               int zchunk, hipStream_t s);

// Interior-only helpers (the boundary shell of dst is never written).
hipError_t launch_scale_copy(float* dst, const float* src, float a, const dims& d, hipStream_t s);
hipError_t launch_zero_f32(float* dst, const dims& d, hipStream_t s);
hipError_t launch_zero_f64(double* dst, const dims& d, hipStream_t s);
// Zero n consecutive floats (whole fields including their shells).
hipError_t launch_zero_span(float* dst, size_t n, hipStream_t s);

}  // namespace stn
