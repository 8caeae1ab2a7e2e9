// Float64 explicit step with the paper's own exp and ln (Sec. 3.3): the
// power of two is synthesised from the bit pattern of the double and only a
// correction polynomial is evaluated, with the coefficients of Table
// tab:coefficients_approx_correction in Estrin's scheme.
//   2^y (eqs. exp_algorithm_1 - exp_algorithm_3; the model passes base-2
//        exponents, so y is the argument itself): y_f = y - floor(y) and the
//        double whose bits are (int64)(2^52 (y - K_exp(y_f)) + 2^52 1023),
//        K_exp(y_f) ~ 1 + y_f - 2^{y_f} of degree 7 (a_0 .. a_7).
//   log2 (eq. ln_approx without its factor ln 2): x = 2^(p - b) (1 + m) from
//        the exponent and mantissa fields, log2 x = (p - b) + K_ln(m),
//        K_ln(m) ~ log2(1 + m) from the table's twelve coefficients b_0 ..
//        b_11 (degree 11; the text says degree 10, but leaving b_11 out
//        costs 2.5e-3 of accuracy).
//   1 - e^{-x} = 1 - 2^{-x log2 e} with the same exp.
// Outside the range the bit synthesis covers, these functions add what the
// paper's formulas leave open: 2^y is 0 below y = -1022 (normal range only)
// and +inf from y = 1024; log2 of 0 is -inf, of a subnormal is taken after
// scaling by 2^54, of a negative number or NaN is NaN.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MSTRUCT_MODEL_NS mstruct_f64paper

namespace MSTRUCT_MODEL_NS {

// K_exp(y_f) in the grouping the paper prints:
// ((a7 y + a6) y^2 + (a5 y + a4)) y^4 + ((a3 y + a2) y^2 + (a1 y + a0))
__device__ __forceinline__ double k_exp(double y) {
    const double a0 = 1.213071811889e-10, a1 = 3.068528102657e-1, a2 = -2.40226342399359e-1,
                 a3 = -5.55053313414954e-2, a4 = -9.6135243288483e-3, a5 = -1.34288475963084e-3,
                 a6 = -1.43131744483589e-4, a7 = -2.1595656126349e-5;
    const double y2 = y * y, y4 = y2 * y2;
    const double hi = fma(fma(a7, y, a6), y2, fma(a5, y, a4));
    const double lo = fma(fma(a3, y, a2), y2, fma(a1, y, a0));
    return fma(hi, y4, lo);
}

// K_ln(m) by Estrin's scheme: pairs, then pairs of pairs with m^2, m^4, m^8
__device__ __forceinline__ double k_ln(double m) {
    const double b0 = 1.84775672096293e-10, b1 = 1.44269504084132, b2 = -0.721347520143005,
                 b3 = 0.480898345526187, b4 = -0.360675000332004, b5 = 0.288048466919235,
                 b6 = -0.235306287368882, b7 = 0.183102904829435, b8 = -0.1209962689793,
                 b9 = 0.0591503811592113, b10 = -0.0181149492489989, b11 = 0.00254488675605743;
    const double m2 = m * m, m4 = m2 * m2, m8 = m4 * m4;
    const double c0 = fma(b1, m, b0), c1 = fma(b3, m, b2), c2 = fma(b5, m, b4);
    const double c3 = fma(b7, m, b6), c4 = fma(b9, m, b8), c5 = fma(b11, m, b10);
    const double d0 = fma(c1, m2, c0), d1 = fma(c3, m2, c2), d2 = fma(c5, m2, c4);
    return fma(d2, m8, fma(d1, m4, d0));
}

__device__ __forceinline__ double fexp2(double y) {
    if (y != y) return y;
    if (!(y < 1024.0)) return __longlong_as_double(0x7ff0000000000000LL);
    if (y < -1022.0) return 0.0;
    const double yf = y - floor(y);
    const double A = 4503599627370496.0;  // 2^52
    return __longlong_as_double((long long)(A * (y - k_exp(yf)) + A * 1023.0));
}

__device__ __forceinline__ double flog2(double x) {
    if (!(x > 0.0)) return x == 0.0 ? __longlong_as_double((long long)0xfff0000000000000ULL) : (x - x) / 0.0;
    if (x == __longlong_as_double(0x7ff0000000000000LL)) return x;
    long long bits = __double_as_longlong(x);
    double e = 0.0;
    if (((bits >> 52) & 0x7ff) == 0) {  // subnormal: scale into the normal range
        bits = __double_as_longlong(x * 18014398509481984.0);  // 2^54
        e = -54.0;
    }
    e += (double)(((bits >> 52) & 0x7ff) - 1023);
    const double m = (double)(bits & 0x000fffffffffffffLL) * (1.0 / 4503599627370496.0);  // [0, 1)
    return e + k_ln(m);
}

__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }

__device__ __forceinline__ double one_minus_exp_neg(double x) { return 1.0 - fexp2(-x * 1.4426950408889634074); }

}  // namespace MSTRUCT_MODEL_NS

#include "step_f64.h"

namespace mstruct {
hipError_t launch_step_f64_paper(const double* Tp, const double* Tn, double* beta, double* as, double* am, int64_t n,
                                 double dt, bool corr_prev, bool mart_assign, hipStream_t st) {
    return mstruct_f64paper::launch_step_f64_impl(Tp, Tn, beta, as, am, n, dt,
                                                  mstruct_f64paper::Readings{corr_prev, mart_assign}, st);
}
}  // namespace mstruct
