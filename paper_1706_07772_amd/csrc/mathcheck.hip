// The FP64 elementary functions of the force terms (terms.h), evaluated on
// device arrays so that their accuracy can be checked against a reference
// over the argument ranges the terms give them.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "terms.h"

namespace rx {

__global__ void k_math_eval(int fn, int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                            double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = x[i];
  double v = 0.0;
  switch (fn) {
    case REAXFF_MATH_EXP: v = exp_f(a); break;
    case REAXFF_MATH_EXP_R: v = exp_r(a); break;
    case REAXFF_MATH_EXP_C: v = exp_c(a); break;
    case REAXFF_MATH_LOG: v = log_f(a); break;
    case REAXFF_MATH_LOG_R: v = log_r(a); break;
    case REAXFF_MATH_POW: v = pow_c(a, y[i]); break;
    case REAXFF_MATH_RCBRT: v = rcbrt_f(a); break;
    case REAXFF_MATH_RCP: v = rcp_f(a); break;
    case REAXFF_MATH_RSQRT: v = rsq_f(a); break;
    default: break;
  }
  out[i] = v;
}

}  // namespace rx

extern "C" int reaxff_math_eval(int32_t fn, int64_t n, const double* x, const double* y, double* out,
                                hipStream_t stream) {
  if (fn < REAXFF_MATH_EXP || fn > REAXFF_MATH_RSQRT || n < 0) return REAXFF_ERR_ARG;
  if (n == 0) return REAXFF_OK;
  if (!x || !out || (fn == REAXFF_MATH_POW && !y)) return REAXFF_ERR_ARG;
  const int bs = 256;
  hipLaunchKernelGGL(rx::k_math_eval, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, stream, fn, n, x, y, out);
  return hipGetLastError() == hipSuccess ? REAXFF_OK : REAXFF_ERR_HIP;
}
