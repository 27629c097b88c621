// Host-side interface of the adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace stn {

// One reverse step m of the leapfrog with c(x):
//   lam2 <- 2 lam1 - lam2 + L8(c lam1)
// (lam1 = lambda_{m+1}, lam2 = lambda_{m+2} on entry and lambda_m on return),
// and, in FP64, g += lambda_{m+2} L8(u_p) + lambda_{m+1} L8(u_c) + lambda_m L8(u_n)
// for the u fields given (u_p = u_{m+1}, u_c = u_m, u_n = u_{m-1}; null
// pointers drop their term, all null leaves g untouched).  w: the five L8 weights.
// mu: the fields hold mu = c * lambda instead (zero boundary shells), the step
// is mu_m = 2 mu_{m+1} - mu_{m+2} + c L8(mu_{m+1}) and the terms use mu.
hipError_t launch_adjoint_step(bool coef_bf16, bool mu, const float* lam1, float* lam2,
                               const void* coef, const float* u_p, const float* u_c,
                               const float* u_n, double* g, const dims& d, const double* w,
                               int zchunk, hipStream_t s);

// Scaled form helpers (interior only): dst = c * src; the final division
// g /= c, g_u0 = mu0 / c, g_um1 = -mu1 / c; and flag = 1 if some |c| is below
// 2^-60 or not finite (flag is cleared first).
hipError_t launch_mul_coef(float* dst, const float* src, bool coef_bf16, const void* coef,
                           const dims& d, hipStream_t s);
hipError_t launch_finish_mu(double* g, float* g_u0, float* g_um1, const float* mu0,
                            const float* mu1, bool coef_bf16, const void* coef, const dims& d,
                            hipStream_t s);
hipError_t launch_coef_check(int* flag, bool coef_bf16, const void* coef, const dims& d,
                             hipStream_t s);

// Adjoint of the variable-coefficient Jacobi kinds 2 (Fig. 1c) and 3 (Fig. 1d).
//
// launch_transpose7: the coefficients W' of the 7-point transpose (interior
// only; dst arrays at element stride dk, src at sk, same storage type), so
// that a forward kind-2 sweep with W' applied to lambda (zero shell) is one
// reverse step lambda_t = A^T lambda_{t+1}.
hipError_t launch_transpose7(void* dst, int64_t dk, const void* src, int64_t sk, bool coef_bf16,
                             const dims& d, hipStream_t s);
// One reverse step of the 25-point stencil: lam0 <- A^T lam1 on the interior
// (lam1 is read on the interior only; the shell of lam0 is not written).
hipError_t launch_adj25_step(bool coef_bf16, const float* lam1, float* lam0, const void* coef,
                             int64_t sk, const dims& d, int zchunk, hipStream_t s);
// Gradient terms of n consecutive steps (1 <= n <= grad_group_max(kind)):
// g_k += sum_i lam[i] * tap_k(u[i]) in FP64, with u[i] = u_s (boundary shell
// included) and lam[i] = lambda_{s+1} for the steps s of the group; the K
// FP64 arrays of g lie at element stride sk.
constexpr int kGradGroupMax = 8;
constexpr int grad_group_max(int kind) { return kind == 2 ? 8 : 6; }
hipError_t launch_jacobi_grad(int kind, int n, const float* const* u, const float* const* lam,
                              double* g, int64_t sk, const dims& d, int zchunk, hipStream_t s);

// Interior-only helpers (the boundary shell of dst is never written).
hipError_t launch_scale_copy(float* dst, const float* src, float a, const dims& d, hipStream_t s);
hipError_t launch_zero_f32(float* dst, const dims& d, hipStream_t s);
hipError_t launch_zero_f64(double* dst, const dims& d, hipStream_t s);
// Zero n consecutive floats (whole fields including their shells).
hipError_t launch_zero_span(float* dst, size_t n, hipStream_t s);

}  // namespace stn
