// Float64 explicit step with the device math library's exp2, log2 and expm1.
#include <hip/hip_runtime.h>

#define MSTRUCT_MODEL_NS mstruct_f64lib

namespace MSTRUCT_MODEL_NS {
__device__ __forceinline__ double fexp2(double x) { return exp2(x); }
__device__ __forceinline__ double flog2(double x) { return log2(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ double one_minus_exp_neg(double x) { return -expm1(-x); }
}  // namespace MSTRUCT_MODEL_NS

#include "step_f64.h"

namespace mstruct {
hipError_t launch_step_f64_library(const double* Tp, const double* Tn, double* beta, double* as, double* am,
                                   int64_t n, double dt, bool corr_prev, bool mart_assign, hipStream_t st) {
    return mstruct_f64lib::launch_step_f64_impl(Tp, Tn, beta, as, am, n, dt,
                                                mstruct_f64lib::Readings{corr_prev, mart_assign}, st);
}
}  // namespace mstruct
