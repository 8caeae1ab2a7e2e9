// Float64 explicit step with exp2 / log2 built from the bit pattern of the
// double (the CPU technique of Sec. 3.3, carried over to test whether it pays
// on the GPU): an integer power of two is written into the exponent field and
// only a short polynomial is evaluated on the reduced argument.
//   2^x: x = n + f with n = rint(x), |f| <= 1/2; 2^f = e^{f ln 2} from its
//        Taylor series to degree 13 (|f ln 2| <= 0.347, remainder < 2^-56);
//        2^n written as exponent bits, in two factors so that results down
//        to the subnormal range are exact.
//   log2: x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s),
//        s = (m - 1)/(m + 1), |s| <= 0.1716, from its series to s^21.
//   1 - e^{-x}: its Taylor series for x < 1/4 (to degree 16), else 1 - 2^{-x log2 e}.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MSTRUCT_MODEL_NS mstruct_f64syn

namespace MSTRUCT_MODEL_NS {

__device__ __forceinline__ double pow2i(int n) {  // 2^n for -1022 <= n <= 1023
    return __longlong_as_double((long long)(n + 1023) << 52);
}

__device__ __forceinline__ double fexp2(double x) {
    if (!(x < 1024.0)) return x != x ? x : __longlong_as_double(0x7ff0000000000000LL);  // NaN or overflow
    if (x < -1075.0) return 0.0;
    const double n = rint(x);
    const double f = (x - n) * 0.6931471805599453094;
    // Taylor coefficients 1/k!, k = 13 .. 0
    double p = 1.6059043836821614599e-10;
    p = fma(f, p, 2.0876756987868098979e-9);
    p = fma(f, p, 2.5052108385441718775e-8);
    p = fma(f, p, 2.7557319223985890653e-7);
    p = fma(f, p, 2.7557319223985890653e-6);
    p = fma(f, p, 2.4801587301587301587e-5);
    p = fma(f, p, 1.9841269841269841270e-4);
    p = fma(f, p, 1.3888888888888888889e-3);
    p = fma(f, p, 8.3333333333333333333e-3);
    p = fma(f, p, 4.1666666666666666667e-2);
    p = fma(f, p, 1.6666666666666666667e-1);
    p = fma(f, p, 0.5);
    p = fma(f, p, 1.0);
    p = fma(f, p, 1.0);
    const int k = (int)n;
    const int k1 = k / 2;
    return p * pow2i(k1) * pow2i(k - k1);
}

__device__ __forceinline__ double flog2(double x) {
    if (!(x > 0.0)) return x == 0.0 ? __longlong_as_double((long long)0xfff0000000000000ULL) : (x - x) / 0.0;
    if (x == __longlong_as_double(0x7ff0000000000000LL)) return x;
    long long bits = __double_as_longlong(x);
    int e = 0;
    if (((bits >> 52) & 0x7ff) == 0) {  // subnormal: scale by 2^54
        x *= 18014398509481984.0;
        bits = __double_as_longlong(x);
        e = -54;
    }
    e += (int)((bits >> 52) & 0x7ff) - 1023;
    double m = __longlong_as_double((bits & 0x000fffffffffffffLL) | 0x3ff0000000000000LL);  // [1, 2)
    if (m > 1.4142135623730950488) {
        m *= 0.5;
        e += 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    // atanh(s) / s = sum s^(2j) / (2j + 1), j = 10 .. 0
    double p = 1.0 / 21.0;
    p = fma(s2, p, 1.0 / 19.0);
    p = fma(s2, p, 1.0 / 17.0);
    p = fma(s2, p, 1.0 / 15.0);
    p = fma(s2, p, 1.0 / 13.0);
    p = fma(s2, p, 1.0 / 11.0);
    p = fma(s2, p, 1.0 / 9.0);
    p = fma(s2, p, 1.0 / 7.0);
    p = fma(s2, p, 1.0 / 5.0);
    p = fma(s2, p, 1.0 / 3.0);
    p = fma(s2, p, 1.0);
    // log2 m = 2 atanh(s) / ln 2
    return fma(2.8853900817779268147 * s, p, (double)e);
}

__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }

__device__ __forceinline__ double one_minus_exp_neg(double x) {
    if (x < 0.25) {
        // x sum (-x)^k / (k+1)!, k = 15 .. 0
        double p = -1.0 / 20922789888000.0;
        p = fma(x, p, 1.0 / 1307674368000.0);
        p = fma(x, p, -1.0 / 87178291200.0);
        p = fma(x, p, 1.0 / 6227020800.0);
        p = fma(x, p, -1.0 / 479001600.0);
        p = fma(x, p, 1.0 / 39916800.0);
        p = fma(x, p, -1.0 / 3628800.0);
        p = fma(x, p, 1.0 / 362880.0);
        p = fma(x, p, -1.0 / 40320.0);
        p = fma(x, p, 1.0 / 5040.0);
        p = fma(x, p, -1.0 / 720.0);
        p = fma(x, p, 1.0 / 120.0);
        p = fma(x, p, -1.0 / 24.0);
        p = fma(x, p, 1.0 / 6.0);
        p = fma(x, p, -0.5);
        p = fma(x, p, 1.0);
        return x * p;
    }
    return 1.0 - fexp2(-x * 1.4426950408889634074);
}

}  // namespace MSTRUCT_MODEL_NS

#include "step_f64.h"

namespace mstruct {
hipError_t launch_step_f64_synth(const double* Tp, const double* Tn, double* beta, double* as, double* am,
                                 int64_t n, double dt, bool corr_prev, bool mart_assign, hipStream_t st) {
    return mstruct_f64syn::launch_step_f64_impl(Tp, Tn, beta, as, am, n, dt,
                                                mstruct_f64syn::Readings{corr_prev, mart_assign}, st);
}
}  // namespace mstruct
