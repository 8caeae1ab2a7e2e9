// The explicit step in float64 (Algorithm 1's loop with the local step of
// Algorithm 2), included by the two float64 translation units after they
// define their double math (see phase_model.h).  40 bytes read and 24 bytes
// written per point.
#pragma once
#include "phase_model.h"

namespace MSTRUCT_MODEL_NS {

__global__ __launch_bounds__(256) void step_f64_kernel(const double* __restrict__ Tp, const double* __restrict__ Tn,
                                                      double* __restrict__ beta, double* __restrict__ as,
                                                      double* __restrict__ am, int64_t n, double dt, Readings rd) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n) return;
    double a = as[g], m = am[g], alo = 0.0, mlo = 0.0;
    const double T0 = Tp[g], T1 = Tn[g];
    const double b = explicit_step<false>(a, m, alo, mlo, T0, alpha_eq(T0), T1, alpha_eq(T1), dt, rd);
    as[g] = a;
    am[g] = m;
    beta[g] = b;
}

inline hipError_t launch_step_f64_impl(const double* Tp, const double* Tn, double* beta, double* as, double* am,
                                       int64_t n, double dt, Readings rd, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(step_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Tp, Tn, beta, as, am,
                       n, dt, rd);
    return hipGetLastError();
}

}  // namespace MSTRUCT_MODEL_NS
