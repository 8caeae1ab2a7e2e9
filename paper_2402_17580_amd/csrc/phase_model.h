// Device (gfx950) implementation of the Ti-6Al-4V phase model of Proell et
// al., arXiv 2402.17580, Sec. 2.2 and Sec. 3.1, in float32.
//
// Transcendentals go to the hardware units: v_exp_f32 / v_log_f32 are base-2,
// so powers a^p (eq. power_exp_log) are exp2(p * log2 a); a = 0 gives
// log2 = -inf and exp2(-inf) = 0, which is the value of the rate factors at
// a zero fraction.  1 - exp(-x) in the Koistinen-Marburger laws uses a
// Taylor polynomial for small x so that the equilibria stay accurate near
// their start temperatures.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mstruct {

// Table 1 / Table 2 / Table 3 of the paper and T_as,reg = 100 K (Sec. 2.2)
constexpr float kTsol = 1878.0f;
constexpr float kTliq = 1928.0f;
constexpr float kTinf = 293.0f;
constexpr float kTasStart = 1273.0f;
constexpr float kTasEnd = 935.0f;
constexpr float kTamStart = 848.0f;
constexpr float kKalphaEq = 0.0068f;
constexpr float kKamEq = 0.00415f;
constexpr float kCas = 2.51f;
constexpr float kCbeta = 11.0f;
constexpr float kK1 = 0.294f;
constexpr float kK2 = 850.0f;
constexpr float kK3 = 0.0337f;
constexpr float kF = 3.8f;
constexpr float kTreg = 100.0f;
constexpr float kXmax = 0.9f;            // maximum alpha fraction
constexpr float kStartupLimit = 1e-15f;  // Appendix A exit test on X~beta * dt
constexpr float kCnEpsAbs = 1e-10f;      // WRMS weights of the implicit scheme (Sec. 3.1)
constexpr float kCnEpsRel = 1e-3f;

// exponents (c -/+ 1)/c of the generalised logistic rates
constexpr float kPa = (kCas - 1.0f) / kCas;
constexpr float kQa = (kCas + 1.0f) / kCas;
constexpr float kPb = (kCbeta - 1.0f) / kCbeta;
constexpr float kQb = (kCbeta + 1.0f) / kCbeta;
constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// 1 - exp(-x) for x >= 0, accurate to a few ulp of the result
__device__ __forceinline__ float one_minus_exp_neg(float x) {
    if (x < 0.25f) {
        // x (1 - x/2 + x^2/6 - x^3/24 + x^4/120 - x^5/720 + x^6/5040)
        float p = fmaf(x, 1.0f / 5040.0f, -1.0f / 720.0f);
        p = fmaf(x, p, 1.0f / 120.0f);
        p = fmaf(x, p, -1.0f / 24.0f);
        p = fmaf(x, p, 1.0f / 6.0f);
        p = fmaf(x, p, -0.5f);
        p = fmaf(x, p, 1.0f);
        return x * p;
    }
    return 1.0f - fexp2(-x * kLog2e);
}

// liquid fraction g(T), eq. liquid_fraction; X_sol = 1 - g
__device__ __forceinline__ float solid_fraction(float T) {
    if (T < kTsol) return 1.0f;
    if (T > kTliq) return 0.0f;
    return 1.0f - (T - kTsol) * (1.0f / (kTliq - kTsol));
}

// X_alpha^eq(T), eq. equilibrium_phase_as
__device__ __forceinline__ float alpha_eq(float T) {
    if (T < kTasEnd) return kXmax;
    if (T > kTasStart) return 0.0f;
    return one_minus_exp_neg(kKalphaEq * (kTasStart - T));
}

// X_alpha_m,0^eq(T), eq. equilibrium_phase_am0 (zero above the martensite start)
__device__ __forceinline__ float am0_eq(float T) {
    if (T < kTinf) return kXmax;
    if (T > kTamStart) return 0.0f;
    return one_minus_exp_neg(kKamEq * (kTamStart - T));
}

// k_alpha_s(T) = k1 / (1 + exp(-k3 (T - k2)))
__device__ __forceinline__ float k_alpha_s(float T) {
    return kK1 * frcp(1.0f + fexp2(-kK3 * kLog2e * (T - kK2)));
}

// Appendix A closed form: fraction X = D xi after dt for
// xi' = kt xi^((c-1)/c) (1-xi)^((c+1)/c) at constant kt.
__device__ __forceinline__ float logistic_step(float X, float D, float kt, float c, float inv_c,
                                               float dt) {
    if (!(D > 0.0f)) return X;
    float xi = fmaxf(X, 0.0f) * frcp(D);
    if (!(xi < 1.0f)) return X;
    float u = fexp2(inv_c * flog2(xi * frcp(1.0f - xi)));  // (xi/(1-xi))^(1/c); 0 at xi = 0
    float w = c * frcp(fmaf(kt, dt, c * u));
    float wc = fexp2(c * flog2(w));  // overflow -> inf -> result 0
    return D * frcp(1.0f + wc);
}

// Diffusive increments over one explicit step (eq. explicit_integration) at
// T^n: beta -> alpha_s, alpha_m -> alpha_s, alpha_s -> beta, with the
// closed-form start from zero-rate states.  X~beta = 0.9 - X_alpha.
__device__ __forceinline__ void diffusive_increment(float a, float m, float Tn, float xeq, float dt,
                                                    float& da, float& dm) {
    float xa = a + m;
    da = 0.0f;
    dm = 0.0f;
    const bool grow = xa < xeq, dissolve = xa > xeq, marten = m > 0.0f;
    if (!(grow | dissolve | marten)) return;
    const float kas = k_alpha_s(Tn);
    const float la = flog2(a);  // -inf at a = 0
    if (grow) {
        if (a > 0.0f) {
            da = dt * kas * fexp2(fmaf(kPa, la, kQa * flog2(xeq - xa)));
        } else {
            const float D = xeq - m;
            if (D > 0.0f) da = logistic_step(0.0f, D, kas * D, kCas, 1.0f / kCas, dt);
        }
    }
    if (marten) {
        const float r2 = kas * fexp2(fmaf(kPa, la, kQa * flog2(m)));
        da = fmaf(dt, r2, da);
        dm = -dt * r2;
    }
    if (dissolve) {
        const float kb = kF * kas;
        const float bt = fmaxf(kXmax - xa, 0.0f);
        if (bt * dt <= kStartupLimit) {
            const float D = kXmax - xeq;
            const float nb = logistic_step(bt, D, D * kb, kCbeta, 1.0f / kCbeta, dt);
            da -= (nb - bt);
        } else {
            da -= dt * kb * fexp2(fmaf(kPb, flog2(bt), kQb * flog2(xa - xeq)));
        }
    }
}

// Correction g(T^{n+1}, m~), eq. explicit_correction: clip at zero, cap the
// alpha total at 0.9 keeping the ratio, alpha_s regularisation above the
// alpha_s start temperature, instantaneous martensite dissolution (eq.
// inst_martensite_dissolution) and formation (eq. inst_martensite_formation,
// never lowering alpha_m), the 0.9 cap again, the solid-fraction cap; returns
// X_beta from the sum rule (eq. beta_post_processing).  xeq = X_alpha^eq(T).
__device__ __forceinline__ float correct(float T, float xeq, float& a_io, float& m_io) {
    float a = fmaxf(a_io, 0.0f), m = fmaxf(m_io, 0.0f);
    float s = a + m;
    if (s > kXmax) {
        const float f = kXmax * frcp(s);
        a *= f;
        m *= f;
    }
    if (T > kTasStart) {
        const float f = fminf(fmaxf((kTasStart + kTreg - T) * (1.0f / kTreg), 0.0f), 1.0f);
        a = fminf(a, kXmax * f);
    }
    if (a + m > xeq) m = fmaxf(xeq - a, 0.0f);
    if (T < kTamStart) m = fmaxf(m, am0_eq(T) * (kXmax - a) * (1.0f / kXmax));
    s = a + m;
    if (s > kXmax) {
        const float f = kXmax * frcp(s);
        a *= f;
        m *= f;
    }
    const float xsol = solid_fraction(T);
    s = a + m;
    if (s > xsol) {
        const float f = (s > 0.0f) ? xsol * frcp(s) : 0.0f;
        a *= f;
        m *= f;
    }
    a_io = a;
    m_io = m;
    return xsol - a - m;
}

// error-free sum: s + e == a + b exactly (Knuth's two-sum)
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// One explicit step on a register state.  With COMPENSATED the Euler
// increments are accumulated in (hi, lo) pairs so that increments below half
// an ulp of the fraction are not lost; any correction that changes a
// fraction resets its lo part.  Returns X_beta^{n+1}.
template <bool COMPENSATED>
__device__ __forceinline__ float explicit_step(float& a, float& m, float& a_lo, float& m_lo, float Tn,
                                               float xeq_n, float Tn1, float xeq_n1, float dt) {
    float da, dm;
    diffusive_increment(a, m, Tn, xeq_n, dt, da, dm);
    float at, mt;
    if (COMPENSATED) {
        two_sum(a, a_lo + da, at, a_lo);
        two_sum(m, m_lo + dm, mt, m_lo);
    } else {
        at = a + da;
        mt = m + dm;
    }
    const float a_before = at, m_before = mt;
    const float beta = correct(Tn1, xeq_n1, at, mt);
    if (COMPENSATED) {
        if (at != a_before) a_lo = 0.0f;
        if (mt != m_before) m_lo = 0.0f;
    }
    a = at;
    m = mt;
    return beta;
}

// Diffusive rate vector [alpha_s', alpha_m'] (eqs. beta_to_alpha_s,
// alpha_m_to_alpha_s, alpha_s_to_beta, split as in eq. diff_inst_split) at a
// temperature with X_alpha^eq = xeq and k_alpha_s = kas; X~beta = 0.9 - X_alpha.
__device__ __forceinline__ void diffusive_rates(float a, float m, float xeq, float kas, float& fa, float& fm) {
    const float xa = a + m;
    const float la = flog2(a);  // -inf at a = 0: the rates that carry a^p vanish
    fa = 0.0f;
    fm = 0.0f;
    if (xa < xeq) fa = kas * fexp2(fmaf(kPa, la, kQa * flog2(xeq - xa)));
    if (m > 0.0f) {
        const float r2 = kas * fexp2(fmaf(kPa, la, kQa * flog2(m)));
        fa += r2;
        fm = -r2;
    }
    if (xa > xeq) {
        const float bt = fmaxf(kXmax - xa, 0.0f);
        fa -= kF * kas * fexp2(fmaf(kPb, flog2(bt), kQb * flog2(xa - xeq)));
    }
}

// One step of the implicit scheme (eqs. implicit_integration,
// implicit_correction): Crank-Nicolson on the diffusive term with g at
// T^{n+1}, solved by the fixed-point iteration of eq. implicit_fp_iteration
// from g(T^{n+1}, m^n).  The iteration stops when the WRMS norm of the
// residual over (alpha_s, alpha_m), weights 1 / (eps_abs + |m_j| eps_rel) of
// the newest iterate, falls below 1, or after max_iter iterations.  A state
// in a start-up regime at T^n (zero rate of a starting transformation) takes
// the explicit step with its Appendix A closed form instead.  With
// COMPENSATED the increment m^{n+1} - m^n is added to (hi, lo) pairs as in
// explicit_step.  Returns the iteration count (0 for a start-up step),
// negated if the stop test failed.
template <bool COMPENSATED>
__device__ __forceinline__ int implicit_step(float& a, float& m, float& a_lo, float& m_lo, float& beta, float Tn,
                                             float Tn1, float dt, int max_iter) {
    const float xeq_n = alpha_eq(Tn), xeq_1 = alpha_eq(Tn1);
    const float xa = a + m;
    if ((xa < xeq_n && !(a > 0.0f)) || (xa > xeq_n && fmaxf(kXmax - xa, 0.0f) * dt <= kStartupLimit)) {
        beta = explicit_step<COMPENSATED>(a, m, a_lo, m_lo, Tn, xeq_n, Tn1, xeq_1, dt);
        return 0;
    }
    const float k_1 = k_alpha_s(Tn1);
    float fa_n, fm_n;
    diffusive_rates(a, m, xeq_n, k_alpha_s(Tn), fa_n, fm_n);
    float ai = a, mi = m, ali = 0.0f, mli = 0.0f;
    beta = correct(Tn1, xeq_1, ai, mi);
    float fa, fm;
    diffusive_rates(ai, mi, xeq_1, k_1, fa, fm);
    const float h = 0.5f * dt;
    int it = 0;
    bool converged = false;
    while (it < max_iter) {
        const float da = h * (fa + fa_n), dm = h * (fm + fm_n);
        float a1, m1, al1 = 0.0f, ml1 = 0.0f;
        if (COMPENSATED) {
            two_sum(a, a_lo + da, a1, al1);
            two_sum(m, m_lo + dm, m1, ml1);
        } else {
            a1 = a + da;
            m1 = m + dm;
        }
        const float a_before = a1, m_before = m1;
        beta = correct(Tn1, xeq_1, a1, m1);
        if (COMPENSATED) {
            if (a1 != a_before) al1 = 0.0f;
            if (m1 != m_before) ml1 = 0.0f;
        }
        float fa1, fm1;
        diffusive_rates(a1, m1, xeq_1, k_1, fa1, fm1);
        const float wa = h * (fa1 - fa) * frcp(fmaf(fabsf(a1), kCnEpsRel, kCnEpsAbs));
        const float wm = h * (fm1 - fm) * frcp(fmaf(fabsf(m1), kCnEpsRel, kCnEpsAbs));
        ai = a1;
        mi = m1;
        ali = al1;
        mli = ml1;
        fa = fa1;
        fm = fm1;
        ++it;
        if (0.5f * fmaf(wa, wa, wm * wm) < 1.0f) {
            converged = true;
            break;
        }
    }
    a = ai;
    m = mi;
    if (COMPENSATED) {
        a_lo = ali;
        m_lo = mli;
    }
    return converged ? it : -it;
}

}  // namespace mstruct
