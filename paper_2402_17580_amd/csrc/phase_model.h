// Device (gfx950) implementation of the Ti-6Al-4V phase model of Proell et
// al., arXiv 2402.17580, Sec. 2.2 and Sec. 3.1, generic in the real type.
//
// float (the hot path): transcendentals go to the hardware units; v_exp_f32 /
// v_log_f32 are base-2, so powers a^p (eq. power_exp_log) are
// exp2(p * log2 a); a = 0 gives log2 = -inf and exp2(-inf) = 0, which is the
// value of the rate factors at a zero fraction.  1 - exp(-x) in the
// Koistinen-Marburger laws uses a Taylor polynomial for small x so that the
// equilibria stay accurate near their start temperatures.
//
// double: the translation unit that instantiates the model in double defines
// fexp2, flog2, frcp and one_minus_exp_neg for double (declared below) before
// use, and sets MSTRUCT_MODEL_NS to a namespace of its own, so that each
// choice of double math is a separate set of functions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef MSTRUCT_MODEL_NS
#define MSTRUCT_MODEL_NS mstruct
#endif

namespace MSTRUCT_MODEL_NS {

// Table 1 / Table 2 / Table 3 of the paper and T_as,reg = 100 K (Sec. 2.2),
// in the model's real type
template <class R>
struct Const {
    static constexpr R Tsol = R(1878.0);
    static constexpr R Tliq = R(1928.0);
    static constexpr R Tinf = R(293.0);
    static constexpr R TasStart = R(1273.0);
    static constexpr R TasEnd = R(935.0);
    static constexpr R TamStart = R(848.0);
    static constexpr R KalphaEq = R(0.0068);
    static constexpr R KamEq = R(0.00415);
    static constexpr R Cas = R(2.51);
    static constexpr R Cbeta = R(11.0);
    static constexpr R K1 = R(0.294);
    static constexpr R K2 = R(850.0);
    static constexpr R K3 = R(0.0337);
    static constexpr R F = R(3.8);
    static constexpr R Treg = R(100.0);
    static constexpr R Xmax = R(0.9);            // maximum alpha fraction
    static constexpr R StartupLimit = R(1e-15);  // Appendix A exit test on X~beta * dt
    static constexpr R CnEpsAbs = R(1e-10);      // WRMS weights of the implicit scheme (Sec. 3.1)
    static constexpr R CnEpsRel = R(1e-3);
    // exponents (c -/+ 1)/c of the generalised logistic rates
    static constexpr R Pa = (Cas - R(1)) / Cas;
    static constexpr R Qa = (Cas + R(1)) / Cas;
    static constexpr R Pb = (Cbeta - R(1)) / Cbeta;
    static constexpr R Qb = (Cbeta + R(1)) / Cbeta;
    static constexpr R Log2e = R(1.4426950408889634);
};

// The two readings of the paper a context can switch (both false: the
// documented defaults).  corr_prev: the explicit correction g at T^n, the
// argument Algorithm 2 passes, instead of T^{n+1} as eq. explicit_correction
// writes it (the implicit scheme corrects at T^{n+1} in both, eq.
// implicit_correction).  mart_assign: eq. inst_martensite_formation's "="
// taken literally, X_am <- X_am^eq below the martensite start, which lowers
// alpha_m on reheating, instead of never lowering it.
struct Readings {
    bool corr_prev;
    bool mart_assign;
};

// float constants used by the kernels
constexpr float kTasStart = Const<float>::TasStart;
constexpr float kTamStart = Const<float>::TamStart;
constexpr float kXmax = Const<float>::Xmax;
constexpr float kLog2e = Const<float>::Log2e;

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fexp2(double x);
__device__ __forceinline__ double flog2(double x);
__device__ __forceinline__ double frcp(double x);

__device__ __forceinline__ float vfma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double vfma(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float vabs(float a) { return fabsf(a); }
__device__ __forceinline__ double vabs(double a) { return fabs(a); }

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
__device__ __forceinline__ double one_minus_exp_neg(double x);

// liquid fraction g(T), eq. liquid_fraction; X_sol = 1 - g
template <class R>
__device__ __forceinline__ R solid_fraction(R T) {
    using C = Const<R>;
    if (T < C::Tsol) return R(1);
    if (T > C::Tliq) return R(0);
    return R(1) - (T - C::Tsol) * (R(1) / (C::Tliq - C::Tsol));
}

// X_alpha^eq(T), eq. equilibrium_phase_as
template <class R>
__device__ __forceinline__ R alpha_eq(R T) {
    using C = Const<R>;
    if (T < C::TasEnd) return C::Xmax;
    if (T > C::TasStart) return R(0);
    return one_minus_exp_neg(C::KalphaEq * (C::TasStart - T));
}

// X_alpha_m,0^eq(T), eq. equilibrium_phase_am0 (zero above the martensite start)
template <class R>
__device__ __forceinline__ R am0_eq(R T) {
    using C = Const<R>;
    if (T < C::Tinf) return C::Xmax;
    if (T > C::TamStart) return R(0);
    return one_minus_exp_neg(C::KamEq * (C::TamStart - T));
}

// k_alpha_s(T) = k1 / (1 + exp(-k3 (T - k2)))
template <class R>
__device__ __forceinline__ R k_alpha_s(R T) {
    using C = Const<R>;
    return C::K1 * frcp(R(1) + fexp2(-C::K3 * C::Log2e * (T - C::K2)));
}

// Appendix A closed form: fraction X = D xi after dt for
// xi' = kt xi^((c-1)/c) (1-xi)^((c+1)/c) at constant kt.
template <class R>
__device__ __forceinline__ R logistic_step(R X, R D, R kt, R c, R inv_c, R dt) {
    if (!(D > R(0))) return X;
    R xi = vmax(X, R(0)) * frcp(D);
    if (!(xi < R(1))) return X;
    R u = fexp2(inv_c * flog2(xi * frcp(R(1) - xi)));  // (xi/(1-xi))^(1/c); 0 at xi = 0
    R w = c * frcp(vfma(kt, dt, c * u));
    R wc = fexp2(c * flog2(w));  // overflow -> inf -> result 0
    return D * frcp(R(1) + wc);
}

// Diffusive increments over one explicit step (eq. explicit_integration) at
// T^n: beta -> alpha_s, alpha_m -> alpha_s, alpha_s -> beta, with the
// closed-form start from zero-rate states.  X~beta = 0.9 - X_alpha.
template <class R>
__device__ __forceinline__ void diffusive_increment(R a, R m, R Tn, R xeq, R dt, R& da, R& dm) {
    using C = Const<R>;
    R xa = a + m;
    da = R(0);
    dm = R(0);
    const bool grow = xa < xeq, dissolve = xa > xeq, marten = m > R(0);
    if (!(grow | dissolve | marten)) return;
    const R kas = k_alpha_s(Tn);
    const R la = flog2(a);  // -inf at a = 0
    if (grow) {
        if (a > R(0)) {
            da = dt * kas * fexp2(vfma(C::Pa, la, C::Qa * flog2(xeq - xa)));
        } else {
            const R D = xeq - m;
            if (D > R(0)) da = logistic_step(R(0), D, kas * D, C::Cas, R(1) / C::Cas, dt);
        }
    }
    if (marten) {
        const R r2 = kas * fexp2(vfma(C::Pa, la, C::Qa * flog2(m)));
        da = vfma(dt, r2, da);
        dm = -dt * r2;
    }
    if (dissolve) {
        const R kb = C::F * kas;
        const R bt = vmax(C::Xmax - xa, R(0));
        if (bt * dt <= C::StartupLimit) {
            const R D = C::Xmax - xeq;
            const R nb = logistic_step(bt, D, D * kb, C::Cbeta, R(1) / C::Cbeta, dt);
            da -= (nb - bt);
        } else {
            da -= dt * kb * fexp2(vfma(C::Pb, flog2(bt), C::Qb * flog2(xa - xeq)));
        }
    }
}

// Correction g(T^{n+1}, m~), eq. explicit_correction: clip at zero, cap the
// alpha total at 0.9 keeping the ratio, alpha_s regularisation above the
// alpha_s start temperature, instantaneous martensite dissolution (eq.
// inst_martensite_dissolution) and formation (eq. inst_martensite_formation,
// never lowering alpha_m), the 0.9 cap again, the solid-fraction cap; returns
// X_beta from the sum rule (eq. beta_post_processing).  xeq = X_alpha^eq(T).
// The correction with its temperature functions given: xeq = X_alpha^eq(T),
// am0 = X_alpha_m,0^eq(T) (used below the martensite start), xsol = 1 - g(T)
// (for iterations at a fixed temperature).
// assign: the literal reading of the formation law (see Readings).
template <class R>
__device__ __forceinline__ R correct_at(R T, R xeq, R am0, R xsol, R& a_io, R& m_io, bool assign = false) {
    using C = Const<R>;
    R a = vmax(a_io, R(0)), m = vmax(m_io, R(0));
    R s = a + m;
    if (s > C::Xmax) {
        const R f = C::Xmax * frcp(s);
        a *= f;
        m *= f;
    }
    if (T > C::TasStart) {
        const R f = vmin(vmax((C::TasStart + C::Treg - T) * (R(1) / C::Treg), R(0)), R(1));
        a = vmin(a, C::Xmax * f);
    }
    if (a + m > xeq) m = vmax(xeq - a, R(0));
    if (T < C::TamStart) {
        const R meq = am0 * (C::Xmax - a) * (R(1) / C::Xmax);
        m = assign ? meq : vmax(m, meq);
    }
    s = a + m;
    if (s > C::Xmax) {
        const R f = C::Xmax * frcp(s);
        a *= f;
        m *= f;
    }
    s = a + m;
    if (s > xsol) {
        const R f = (s > R(0)) ? xsol * frcp(s) : R(0);
        a *= f;
        m *= f;
    }
    a_io = a;
    m_io = m;
    return xsol - a - m;
}

template <class R>
__device__ __forceinline__ R correct(R T, R xeq, R& a_io, R& m_io, bool assign = false) {
    return correct_at(T, xeq, T < Const<R>::TamStart ? am0_eq(T) : R(0), solid_fraction(T), a_io, m_io, assign);
}

// A fully stable-alpha state (X_alpha_s = 0.9, no martensite) is a fixed point
// of the update while T^n and T^{n+1} stay below the alpha_s -> beta end
// temperature: X_alpha = X_alpha^eq = 0.9 there, so every diffusive rate is
// zero, and the correction leaves it alone (the formation law raises alpha_m
// to at most X_alpha_m,0^eq (0.9 - X_alpha_s) / 0.9 = 0).  Steps of such a
// state return it unchanged without evaluating the model; the result is the
// same as that of the full evaluation, bit for bit, in either reading of
// Readings (g at T^n or T^{n+1}, both below 935 K; formation sets alpha_m to
// 0 either way).  Away from the laser most of a part is in this state.
template <class R>
__device__ __forceinline__ bool at_rest(R a, R m, R Tn, R Tn1) {
    using C = Const<R>;
    return a == C::Xmax && m == R(0) && Tn < C::TasEnd && Tn1 < C::TasEnd;
}

// error-free sum: s + e == a + b exactly (Knuth's two-sum)
template <class R>
__device__ __forceinline__ void two_sum(R a, R b, R& s, R& e) {
    s = a + b;
    const R bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// One explicit step on a register state.  With COMPENSATED the Euler
// increments are accumulated in (hi, lo) pairs so that increments below half
// an ulp of the fraction are not lost; any correction that changes a
// fraction resets its lo part.  Returns X_beta^{n+1} (the sum rule at the
// correction's temperature).  A state at rest is returned as it is: with
// m == 0 its lo part is 0, and re-adding the (hi, lo) pair of a previous
// two-sum reproduces it, so the full step would not change it either.
template <bool COMPENSATED, class R>
__device__ __forceinline__ R explicit_step(R& a, R& m, R& a_lo, R& m_lo, R Tn, R xeq_n, R Tn1, R xeq_n1, R dt,
                                           Readings rd = Readings{false, false}) {
    if (at_rest(a, m, Tn, Tn1)) return R(1) - a - m;  // X_sol = 1 below T_as,end
    R da, dm;
    diffusive_increment(a, m, Tn, xeq_n, dt, da, dm);
    R at, mt;
    if (COMPENSATED) {
        two_sum(a, a_lo + da, at, a_lo);
        two_sum(m, m_lo + dm, mt, m_lo);
    } else {
        at = a + da;
        mt = m + dm;
    }
    const R a_before = at, m_before = mt;
    const R beta = rd.corr_prev ? correct(Tn, xeq_n, at, mt, rd.mart_assign)
                                : correct(Tn1, xeq_n1, at, mt, rd.mart_assign);
    if (COMPENSATED) {
        if (at != a_before) a_lo = R(0);
        if (mt != m_before) m_lo = R(0);
    }
    a = at;
    m = mt;
    return beta;
}

// Diffusive rate vector [alpha_s', alpha_m'] (eqs. beta_to_alpha_s,
// alpha_m_to_alpha_s, alpha_s_to_beta, split as in eq. diff_inst_split) at a
// temperature with X_alpha^eq = xeq and k_alpha_s = kas; X~beta = 0.9 - X_alpha.
template <class R>
__device__ __forceinline__ void diffusive_rates(R a, R m, R xeq, R kas, R& fa, R& fm) {
    using C = Const<R>;
    const R xa = a + m;
    const R la = flog2(a);  // -inf at a = 0: the rates that carry a^p vanish
    fa = R(0);
    fm = R(0);
    if (xa < xeq) fa = kas * fexp2(vfma(C::Pa, la, C::Qa * flog2(xeq - xa)));
    if (m > R(0)) {
        const R r2 = kas * fexp2(vfma(C::Pa, la, C::Qa * flog2(m)));
        fa += r2;
        fm = -r2;
    }
    if (xa > xeq) {
        const R bt = vmax(C::Xmax - xa, R(0));
        fa -= C::F * kas * fexp2(vfma(C::Pb, flog2(bt), C::Qb * flog2(xa - xeq)));
    }
}

// One step of the implicit scheme: Crank-Nicolson on the diffusive term
// (eq. implicit_integration) with the correction g at T^{n+1} (eq.
// implicit_correction).  The step's result is the fixed point of eq.
// implicit_fp_iteration,
//   m_(i) = g(T^{n+1}, m^n + dt/2 [f(T^n, m^n) + f(T^{n+1}, m_(i-1))]),
// taken from m_(0) = g(T^{n+1}, m^n) (reading R12); it is accepted at the
// first i >= 1 where the WRMS norm of the equation's residual at m_(i),
// dt/2 [f(T^{n+1}, m_(i)) - f(T^{n+1}, m_(i-1))] over (alpha_s, alpha_m)
// with weights 1 / (eps_abs + |m_(i),j| eps_rel), falls below 1, or at
// i = max_iter.  A state in a start-up regime at T^n (zero rate of a
// starting transformation) takes the explicit step with its Appendix A
// closed form instead.  With COMPENSATED the increment over m^n is added to
// (hi, lo) pairs as in explicit_step.  Returns the number of iterations
// (0 for a start-up step), negated if the stop test failed.  A state at rest
// converges in the first iteration with zero rates and is returned as it is
// (count 1).  assign: see Readings.
template <bool COMPENSATED, class R>
__device__ __forceinline__ int implicit_step(R& a, R& m, R& a_lo, R& m_lo, R& beta, R Tn, R Tn1, R dt,
                                             int max_iter, bool assign = false) {
    using C = Const<R>;
    if (at_rest(a, m, Tn, Tn1)) {
        beta = R(1) - a - m;
        return 1;
    }
    const R xeq_n = alpha_eq(Tn), xeq_1 = alpha_eq(Tn1);
    const R xa = a + m;
    // (the alpha_s -> beta start needs D = 0.9 - X_alpha^eq > 0: below the
    // alpha_s -> beta end temperature X_alpha > X_alpha^eq = 0.9 is rounding)
    if ((xa < xeq_n && !(a > R(0))) ||
        (xa > xeq_n && xeq_n < C::Xmax && vmax(C::Xmax - xa, R(0)) * dt <= C::StartupLimit)) {
        beta = explicit_step<COMPENSATED>(a, m, a_lo, m_lo, Tn, xeq_n, Tn1, xeq_1, dt, Readings{false, assign});
        return 0;
    }
    // functions of T^{n+1}, fixed over the iteration, and f(T^n, m^n)
    const R k_1 = k_alpha_s(Tn1);
    const R am0_1 = Tn1 < C::TamStart ? am0_eq(Tn1) : R(0), xsol_1 = solid_fraction(Tn1);
    R fa_n, fm_n;
    diffusive_rates(a, m, xeq_n, k_alpha_s(Tn), fa_n, fm_n);
    const R h = R(0.5) * dt;
    R a_i = a, m_i = m, alo_i = a_lo, mlo_i = m_lo;  // m_(i)
    R fa_p = R(0), fm_p = R(0);                       // f(T^{n+1}, m_(i-1))
    for (int i = 0;; ++i) {
        // m^n plus the Crank-Nicolson increment (none for m_(0)), then g
        const R da = i > 0 ? h * (fa_p + fa_n) : R(0), dm = i > 0 ? h * (fm_p + fm_n) : R(0);
        R a1, m1, alo1 = R(0), mlo1 = R(0);
        if (COMPENSATED) {
            two_sum(a, a_lo + da, a1, alo1);
            two_sum(m, m_lo + dm, m1, mlo1);
        } else {
            a1 = a + da;
            m1 = m + dm;
        }
        const R a_before = a1, m_before = m1;
        beta = correct_at(Tn1, xeq_1, am0_1, xsol_1, a1, m1, assign);
        if (COMPENSATED) {
            if (a1 != a_before) alo1 = R(0);
            if (m1 != m_before) mlo1 = R(0);
        }
        R fa1, fm1;
        diffusive_rates(a1, m1, xeq_1, k_1, fa1, fm1);
        a_i = a1;
        m_i = m1;
        alo_i = alo1;
        mlo_i = mlo1;
        if (i > 0) {
            const R wa = h * (fa1 - fa_p) * frcp(vfma(vabs(a1), C::CnEpsRel, C::CnEpsAbs));
            const R wm = h * (fm1 - fm_p) * frcp(vfma(vabs(m1), C::CnEpsRel, C::CnEpsAbs));
            const bool converged = R(0.5) * vfma(wa, wa, wm * wm) < R(1);
            if (converged || i >= max_iter) {
                a = a_i;
                m = m_i;
                if (COMPENSATED) {
                    a_lo = alo_i;
                    m_lo = mlo_i;
                }
                return converged ? i : -i;
            }
        }
        fa_p = fa1;
        fm_p = fm1;
    }
}

// ---------------------------------------------------------------------------
// Tracked shifted beta fraction (Appendix A).  When the alpha_s -> beta
// transformation starts, X~beta = 0.9 - X_alpha is far below what X_beta =
// 0.1 + X~beta, or X_alpha_s near 0.9, resolves in float32 (and its early
// values, e.g. 1e-80 after one microsecond at 1200 K, are below the float32
// range), so the paper keeps it apart.  An optional float64 value per point
// carries it while the point is in that regime: no martensite, dissolution at
// T^n (X~beta below D = 0.9 - X_alpha^eq) and X~beta below kTrackMax, above
// which alpha_s resolves it to 1.2e-4 relative.  NaN: nothing is tracked;
// X~beta then follows from the fractions.  The regime's only diffusive rate
// is alpha_s -> beta, so the step is written on X~beta alone, in float64:
// the closed form while X~beta dt is at most 1e-15, then Euler (or
// Crank-Nicolson) on X~beta.  alpha_s = 0.9 - X~beta is stored as a float
// (hi, lo) pair in the compensated kernels, which hands the value over
// exactly when tracking ends.  0.9 is the float model's cap throughout.
// (Float only: the float64 model keeps X~beta in its fractions.)
// ---------------------------------------------------------------------------
constexpr double kTrackMax = 0x1p-12;

__device__ __forceinline__ double track_none() { return __builtin_nan(""); }

// the side value as loaded with the fractions: kept if it agrees with them
// (no martensite, 0.9 - alpha_s within 0.6 ulp of 0.9 of it), NaN otherwise
__device__ __forceinline__ double track_check(double xb, float a, float m) {
    const double d = (double)(Const<float>::Xmax - a) - xb;
    return (m == 0.0f && fabs(d) <= 3.6e-8) ? xb : track_none();
}

// float64 forms of the functions the tracked step needs
__device__ __forceinline__ double alpha_eq_f64(double T) {
    if (T < 935.0) return (double)Const<float>::Xmax;
    if (T > 1273.0) return 0.0;
    return -expm1(-0.0068 * (1273.0 - T));
}
__device__ __forceinline__ double k_beta_f64(double T) {  // f k_alpha_s(T)
    return 3.8 * 0.294 / (1.0 + exp(-0.0337 * (T - 850.0)));
}
// d X~beta / dt = k_b X~beta^((c-1)/c) (D - X~beta)^((c+1)/c), c = 11
__device__ __forceinline__ double beta_rate_f64(double x, double D, double kb) {
    return x < D ? kb * pow(x, 10.0 / 11.0) * pow(D - x, 12.0 / 11.0) : 0.0;
}
// Appendix A closed form from X~beta = x over dt at constant k~ = D k_b
__device__ __forceinline__ double beta_startup_f64(double x, double D, double kb, double dt) {
    const double xi = x / D;
    const double u = pow(xi / (1.0 - xi), 1.0 / 11.0);
    const double w = 11.0 / (D * kb * dt + 11.0 * u);
    return D / (1.0 + pow(w, 11.0));
}

// X~beta if the point is in the tracked regime at T^n (D > 0), else false
__device__ __forceinline__ bool track_regime(float a, float m, double xb, double D, double& bt) {
    bt = (xb == xb) ? xb : (double)fmaxf(Const<float>::Xmax - (a + m), 0.0f);
    return m == 0.0f && bt < D && bt < kTrackMax;
}

// alpha_s = 0.9 - X~beta after a tracked step, then g at Tc (T^{n+1}, or
// T^n with Readings::corr_prev); tracking goes on if g left the state alone
// and X~beta stays below kTrackMax
template <bool COMPENSATED>
__device__ __forceinline__ float track_finish(float& a, float& m, float& a_lo, float& m_lo, double& xb, double bn,
                                              float Tc, float xeq_c, bool assign) {
    const double av = (double)Const<float>::Xmax - bn;
    float at = (float)av;
    const float lo = (float)(av - (double)at);
    float mt = 0.0f;
    const float a_before = at;
    const float beta = correct(Tc, xeq_c, at, mt, assign);
    const bool kept = at == a_before && mt == 0.0f;
    xb = (kept && bn < kTrackMax) ? bn : track_none();
    a = at;
    m = mt;
    a_lo = (COMPENSATED && kept) ? lo : 0.0f;
    m_lo = 0.0f;
    return beta;
}

// explicit_step with the tracked X~beta
template <bool COMPENSATED>
__device__ __forceinline__ float explicit_step_tracked(float& a, float& m, float& a_lo, float& m_lo, double& xb,
                                                       float Tn, float xeq_n, float Tn1, float xeq_n1, float dt,
                                                       Readings rd = Readings{false, false}) {
    double bt;
    const double D = (double)Const<float>::Xmax - alpha_eq_f64(Tn);
    if (at_rest(a, m, Tn, Tn1) || !track_regime(a, m, xb, D, bt)) {
        xb = track_none();
        return explicit_step<COMPENSATED>(a, m, a_lo, m_lo, Tn, xeq_n, Tn1, xeq_n1, dt, rd);
    }
    const double kb = k_beta_f64(Tn), h = dt;
    const double bn = bt * h <= 1e-15 ? beta_startup_f64(bt, D, kb, h) : bt + h * beta_rate_f64(bt, D, kb);
    return rd.corr_prev ? track_finish<COMPENSATED>(a, m, a_lo, m_lo, xb, bn, Tn, xeq_n, rd.mart_assign)
                        : track_finish<COMPENSATED>(a, m, a_lo, m_lo, xb, bn, Tn1, xeq_n1, rd.mart_assign);
}

// implicit_step with the tracked X~beta: the start-up takes the tracked
// explicit step; after it, Crank-Nicolson on X~beta with the same fixed-point
// iteration and WRMS stop (the alpha_m residual is zero).  If g could act on
// the state at T^{n+1} (below the martensite start or above the alpha_s
// start), the value is handed over and the ordinary step is taken.
template <bool COMPENSATED>
__device__ __forceinline__ int implicit_step_tracked(float& a, float& m, float& a_lo, float& m_lo, double& xb,
                                                     float& beta, float Tn, float Tn1, float dt, int max_iter,
                                                     bool assign = false) {
    using C = Const<float>;
    double bt;
    const double D = (double)C::Xmax - alpha_eq_f64(Tn);
    if (at_rest(a, m, Tn, Tn1) || !track_regime(a, m, xb, D, bt)) {
        xb = track_none();
        return implicit_step<COMPENSATED>(a, m, a_lo, m_lo, beta, Tn, Tn1, dt, max_iter, assign);
    }
    if (bt * (double)dt <= 1e-15) {
        xb = bt;
        beta = explicit_step_tracked<COMPENSATED>(a, m, a_lo, m_lo, xb, Tn, alpha_eq(Tn), Tn1, alpha_eq(Tn1), dt,
                                                  Readings{false, assign});
        return 0;
    }
    if (!(Tn1 >= C::TamStart && Tn1 <= C::TasStart)) {
        const double av = (double)C::Xmax - bt;
        a = (float)av;
        a_lo = COMPENSATED ? (float)(av - (double)a) : 0.0f;
        xb = track_none();
        return implicit_step<COMPENSATED>(a, m, a_lo, m_lo, beta, Tn, Tn1, dt, max_iter, assign);
    }
    const double D1 = (double)C::Xmax - alpha_eq_f64(Tn1), kb1 = k_beta_f64(Tn1);
    const double f_n = beta_rate_f64(bt, D, k_beta_f64(Tn));
    const double h = 0.5 * (double)dt;
    double x = bt, f = beta_rate_f64(bt, D1, kb1);  // g(T^{n+1}, m^n) leaves the state alone here
    int it = 0;
    bool converged = false;
    while (it < max_iter) {
        const double x1 = bt + h * (f_n + f);
        const double f1 = beta_rate_f64(x1, D1, kb1);
        const double w = h * (f1 - f) / ((double)C::CnEpsAbs + (double)C::CnEpsRel * fabs((double)C::Xmax - x1));
        x = x1;
        f = f1;
        ++it;
        if (0.5 * w * w < 1.0) {
            converged = true;
            break;
        }
    }
    beta = track_finish<COMPENSATED>(a, m, a_lo, m_lo, xb, x, Tn1, alpha_eq(Tn1), assign);
    return converged ? it : -it;
}

}  // namespace MSTRUCT_MODEL_NS
