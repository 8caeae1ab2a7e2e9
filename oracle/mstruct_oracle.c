/*
 * FP64 CPU oracle for the scan-resolved Ti-6Al-4V phase update.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the HIP library.
 *
 * Everything is double precision with the C library's transcendentals.
 * Each function cites the passage of Proell et al., "A highly efficient
 * computational approach for part-scale microstructure predictions in
 * Ti-6Al-4V additive manufacturing" (arXiv 2402.17580) that it follows.
 *
 * Readings taken where the paper is silent or garbled:
 *   R1  third case of the martensite pseudo-equilibrium is "0 above the
 *       martensite start temperature" (the printed bound names the alpha_s
 *       start temperature, which would leave (848, 1273] undefined).
 *   R2  the alpha_s regularisation applies for every T above the alpha_s start
 *       temperature, with the linear factor clamped to [0, 1].
 *   R3  the explicit correction g is evaluated at T^{n+1} (eq.
 *       explicit_correction), rates at T^n (eq. explicit_integration).
 *   R4  instantaneous martensite formation never lowers alpha_m:
 *       X_am <- max(X_am, X_am^eq) below the martensite start temperature.
 *   R3 and R4 are the defaults of two switches (orc_set_readings): the
 *   explicit correction at T^n (the argument Algorithm 2 passes) instead of
 *   T^{n+1}, and the formation law's "=" taken literally (X_am <- X_am^eq,
 *   which lowers alpha_m on reheating below the martensite start).
 *   R5  order inside g: clip at 0, cap alpha at 0.9 keeping the ratio,
 *       regularisation, martensite dissolution, martensite formation, the
 *       0.9 cap again (formation can overshoot it just above T_inf), the
 *       solid-fraction cap, beta from the sum rule.
 *   R6  alpha_s -> beta start-up (Appendix A) is used while
 *       X_alpha > X_alpha^eq and X~beta * dt <= 1e-15 (dt in seconds), with
 *       T held at T^n over the step; X~beta is carried as its own state and,
 *       while the closed form is in use, is authoritative: alpha_s is set to
 *       X_sol - 0.1 - X~beta - X_am (not accumulated from increments, which
 *       float64 rounds at 1.1e-16 each while they are near 1e-15).
 *   R7  beta -> alpha_s start-up (cited to an absent reference) uses the same
 *       generalised-logistic closed form with X_am frozen:
 *       D' = X_alpha^eq - X_am, k~ = k_as D', c = c_as, from X_as = 0.
 *   R8  when D <= 0 (or the start-up ratio is >= 1) no start-up change.
 *   R9  temperature: switched moving point source on a semi-infinite body
 *       (not part of the paper, which uses an FEM heat solve); the window of
 *       superposed tracks is the last `window` tracks with t_on <= t + 1e-12 s.
 *   R12 implicit scheme: the fixed-point iteration starts from
 *       g(T^{n+1}, m^n), as the implicit algorithm does (the iteration's
 *       equation writes m^n; both reach the same fixed point).
 *   R13 the WRMS norm runs over the two components (alpha_s, alpha_m) without
 *       a square root (the test "< 1" is unaffected), with weights from the
 *       absolute value of the newest iterate; at most max_iter iterations.
 *   R14 a state in a start-up regime at T^n takes the explicit step with its
 *       closed form, since the paper initiates diffusion with the closed form
 *       in both schemes; the alpha_s -> beta start counts only where its
 *       closed form can act (D > 0, i.e. above the alpha_s -> beta end
 *       temperature).
 *   R15 subcycling: a step longer than dt_sub is split into the fewest equal
 *       substeps not longer than dt_sub, with T linear in time.
 *   R16 a switched-off track is the difference of two moving sources that
 *       share a virtual current position beyond the end point; its field is
 *       smooth there but the closed form is 0/0 at it, so within 0.5 um of
 *       that position it is evaluated 0.5 um below it (the clamp applies
 *       only near a switched-on source).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- Table 1 (thermal) and Tables 2-3 (microstructure) of the paper ---- */
static const double T_SOLIDUS = 1878.0;  /* T_s  [K] */
static const double T_LIQUIDUS = 1928.0; /* T_l  [K] */
static const double T_AMBIENT = 293.0;   /* T_inf [K] */
static const double T_AS_START = 1273.0; /* upper end of beta->alpha_s range [K] */
static const double T_AS_END = 935.0;    /* lower end of beta->alpha_s range [K] */
static const double T_AM_START = 848.0;  /* martensite start [K] */
static const double K_ALPHA_EQ = 0.0068; /* [1/K] */
static const double K_AM_EQ = 0.00415;   /* [1/K] */
static const double C_AS = 2.51;
static const double C_BETA = 11.0;
static const double K1 = 0.294;          /* [1/s] */
static const double K2 = 850.0;          /* [K]   */
static const double K3 = 0.0337;         /* [1/K] */
static const double F_BETA = 3.8;
static const double T_AS_REG = 100.0;    /* regularisation width chosen in Sec. 2.2 [K] */
static const double X_ALPHA_MAX = 0.9;   /* maximum alpha fraction (first case of X_alpha^eq) */
static const double STARTUP_LIMIT = 1e-15; /* Appendix A exit criterion on X~beta * dt */

/* the readings of the paper that can be switched (0: the defaults R3, R4) */
static int g_correction_prev = 0;  /* 1: explicit correction at T^n */
static int g_martensite_assign = 0; /* 1: X_am <- X_am^eq below the martensite start */

void orc_set_readings(int correction_prev, int martensite_assign)
{
    g_correction_prev = correction_prev != 0;
    g_martensite_assign = martensite_assign != 0;
}

int orc_get_readings(void)
{
    return g_correction_prev | (g_martensite_assign << 1);
}

int orc_constants(double *out, int n)
{
    const double c[] = {T_SOLIDUS, T_LIQUIDUS, T_AMBIENT, T_AS_START, T_AS_END,
                        T_AM_START, K_ALPHA_EQ, K_AM_EQ, C_AS, C_BETA, K1, K2, K3,
                        F_BETA, T_AS_REG, X_ALPHA_MAX, STARTUP_LIMIT};
    int m = (int)(sizeof(c) / sizeof(c[0]));
    for (int i = 0; i < n && i < m; ++i) out[i] = c[i];
    return m;
}

/* ---------------- model functions (Sec. 2.1, 2.2) ---------------- */

/* liquid fraction g(T), eq. liquid_fraction; X_sol = 1 - g (Sec. 2.2) */
double orc_liquid_fraction(double T)
{
    if (T < T_SOLIDUS) return 0.0;
    if (T > T_LIQUIDUS) return 1.0;
    return (T - T_SOLIDUS) / (T_LIQUIDUS - T_SOLIDUS);
}

/* stable alpha equilibrium, eq. equilibrium_phase_as (Koistinen-Marburger) */
double orc_alpha_eq(double T)
{
    if (T < T_AS_END) return X_ALPHA_MAX;
    if (T > T_AS_START) return 0.0;
    return -expm1(-K_ALPHA_EQ * (T_AS_START - T));
}

/* martensite pseudo-equilibrium, eq. equilibrium_phase_am0 (reading R1) */
double orc_am0_eq(double T)
{
    if (T < T_AMBIENT) return X_ALPHA_MAX;
    if (T > T_AM_START) return 0.0;
    return -expm1(-K_AM_EQ * (T_AM_START - T));
}

/* diffusion rate constant k_alpha_s(T) (Sec. 2.2, after eq. alpha_s_to_beta) */
double orc_k_as(double T)
{
    return K1 / (1.0 + exp(-K3 * (T - K2)));
}

/* the three diffusive rates at (T, state), eqs. beta_to_alpha_s,
 * alpha_m_to_alpha_s, alpha_s_to_beta.  xbt is X~beta = 0.9 - X_alpha, the
 * shifted beta fraction of Appendix A, used for the (0.9 - X_alpha) factor. */
void orc_rates(double as, double am, double xbt, double T, double *r1, double *r2, double *r3)
{
    const double pa = (C_AS - 1.0) / C_AS, qa = (C_AS + 1.0) / C_AS;
    const double pb = (C_BETA - 1.0) / C_BETA, qb = (C_BETA + 1.0) / C_BETA;
    double xa = as + am, xeq = orc_alpha_eq(T), kas = orc_k_as(T);
    *r1 = (xa < xeq) ? kas * pow(as, pa) * pow(xeq - xa, qa) : 0.0;
    *r2 = (am > 0.0) ? kas * pow(as, pa) * pow(am, qa) : 0.0;
    *r3 = (xa > xeq) ? F_BETA * kas * pow(xbt > 0.0 ? xbt : 0.0, pb) * pow(xa - xeq, qb) : 0.0;
}

/* generalised-logistic closed-form step (Appendix A, eq. analytical_solution_beta):
 * for xi' = k~ xi^((c-1)/c) (1-xi)^((c+1)/c) at constant k~, from xi_n after dt,
 * returned as the fraction D * xi_{n+1} given X = D * xi_n. */
double orc_logistic_step(double X, double D, double kt, double c, double dt)
{
    if (!(D > 0.0)) return X;
    double xi = (X > 0.0 ? X : 0.0) / D;
    if (!(xi < 1.0)) return X;
    double u = pow(xi / (1.0 - xi), 1.0 / c);
    double w = c / (kt * dt + c * u);
    return D / (1.0 + pow(w, c));
}

/* correction g(T, m) of eq. explicit_correction with the instantaneous
 * martensite formation / dissolution (eqs. inst_martensite_formation,
 * inst_martensite_dissolution), the alpha_s regularisation and the continuity
 * constraints (eqs. phase_continuity_*), in the order of reading R5.  Returns
 * X_beta from eq. beta_post_processing. */
double orc_correct(double T, double *as_, double *am_)
{
    double a = *as_, m = *am_;
    /* clip negative fractions to zero */
    if (a < 0.0) a = 0.0;
    if (m < 0.0) m = 0.0;
    /* total alpha above 0.9: scale both keeping the ratio */
    double s = a + m;
    if (s > X_ALPHA_MAX) {
        double f = X_ALPHA_MAX / s;
        a *= f;
        m *= f;
    }
    /* alpha_s regularisation above the alpha_s start temperature (R2) */
    if (T > T_AS_START) {
        double f = (T_AS_START + T_AS_REG - T) / T_AS_REG;
        if (f < 0.0) f = 0.0;
        if (f > 1.0) f = 1.0;
        double cap = X_ALPHA_MAX * f;
        if (a > cap) a = cap;
    }
    /* instantaneous martensite dissolution on heating */
    double xeq = orc_alpha_eq(T);
    if (a + m > xeq) {
        m = xeq - a;
        if (m < 0.0) m = 0.0;
    }
    /* instantaneous martensite formation below the martensite start (R4),
     * towards the corrected pseudo-equilibrium of eq. equilibrium_phase_am;
     * with the literal reading of eq. inst_martensite_formation alpha_m is
     * set to it, also where that lowers it */
    if (T < T_AM_START) {
        double meq = orc_am0_eq(T) * (X_ALPHA_MAX - a) / X_ALPHA_MAX;
        if (m < meq || g_martensite_assign) m = meq;
    }
    /* the pseudo-equilibrium can exceed 0.9 just above T_inf: cap again */
    s = a + m;
    if (s > X_ALPHA_MAX) {
        double f = X_ALPHA_MAX / s;
        a *= f;
        m *= f;
    }
    /* solid fraction: alpha cannot exceed X_sol */
    double xsol = 1.0 - orc_liquid_fraction(T);
    if (a + m > xsol) {
        double f = xsol / (a + m);
        a *= f;
        m *= f;
    }
    *as_ = a;
    *am_ = m;
    return xsol - a - m;
}

/* one explicit step (eqs. explicit_integration, explicit_correction) for one
 * point; the start of diffusion from zero-rate states follows Sec. 3.1 and
 * Appendix A (readings R6-R8).  State: alpha_s, alpha_m, beta, X~beta.  The
 * correction is taken at Tc (T^{n+1}, or T^n with the switched reading R3). */
static void step_at(double *as_, double *am_, double *b_, double *bt_, double Tn, double Tc, double dt)
{
    const double pa = (C_AS - 1.0) / C_AS, qa = (C_AS + 1.0) / C_AS;
    const double pb = (C_BETA - 1.0) / C_BETA, qb = (C_BETA + 1.0) / C_BETA;
    double as = *as_, am = *am_, bt = *bt_;
    double xa = as + am;
    double xeq = orc_alpha_eq(Tn);
    double kas = orc_k_as(Tn);
    double kb = F_BETA * kas;
    double das = 0.0, dam = 0.0;
    int startup_beta = 0;
    double bt_new = bt;

    /* beta -> alpha_s */
    if (xa < xeq) {
        if (as > 0.0) {
            das += dt * kas * pow(as, pa) * pow(xeq - xa, qa);
        } else {
            /* zero-rate start: closed form from X_as = 0 (R7) */
            double D = xeq - am;
            if (D > 0.0) das += orc_logistic_step(0.0, D, kas * D, C_AS, dt);
        }
    }
    /* alpha_m -> alpha_s */
    if (am > 0.0) {
        double r2 = kas * pow(as, pa) * pow(am, qa);
        das += dt * r2;
        dam -= dt * r2;
    }
    /* alpha_s -> beta */
    if (xa > xeq) {
        double btp = bt > 0.0 ? bt : 0.0;
        if (btp * dt <= STARTUP_LIMIT) {
            /* Appendix A closed form on the shifted beta fraction (R6) */
            double D = X_ALPHA_MAX - xeq;
            double nb = orc_logistic_step(btp, D, D * kb, C_BETA, dt);
            if (nb != btp) {
                bt_new = nb;
                startup_beta = 1;
            }
        } else {
            das -= dt * kb * pow(btp, pb) * pow(xa - xeq, qb);
        }
    }

    /* forward Euler towards the intermediate state, then the correction;
     * while the start-up form is in use X~beta is authoritative and alpha_s
     * follows from it (R6): X_alpha = 0.9 - X~beta, alpha_m as updated */
    double m = am + dam;
    double a = startup_beta ? X_ALPHA_MAX - bt_new - m : as + das;
    double a_t = a, m_t = m;
    double b = orc_correct(Tc, &a, &m);

    /* X~beta stays authoritative while the start-up form is in use and the
     * correction left the state alone; otherwise it follows the sum rule */
    if (startup_beta && a == a_t && m == m_t)
        bt = bt_new;
    else
        bt = X_ALPHA_MAX - (a + m);
    *as_ = a;
    *am_ = m;
    *b_ = b;
    *bt_ = bt;
}

void orc_step(double *as_, double *am_, double *b_, double *bt_, double Tn, double Tn1, double dt)
{
    step_at(as_, am_, b_, bt_, Tn, g_correction_prev ? Tn : Tn1, dt);
}

void orc_step_n(int64_t n, double *as, double *am, double *b, double *bt,
                const double *Tn, const double *Tn1, double dt)
{
    for (int64_t i = 0; i < n; ++i) orc_step(&as[i], &am[i], &b[i], &bt[i], Tn[i], Tn1[i], dt);
}

/* ---------------- implicit scheme (Sec. 3.1, eqs. implicit_integration,
 * implicit_correction, implicit_fp_iteration and the WRMS stop; the
 * implicit algorithm of Sec. 3.2; readings R12-R15) ---------------- */

/* diffusive part of the rate vector m' = [alpha_s', alpha_m'] (eq.
 * diff_inst_split) at (T, state), X~beta taken as 0.9 - X_alpha */
static void diff_rates(double as, double am, double T, double *fa, double *fm)
{
    double r1, r2, r3;
    orc_rates(as, am, X_ALPHA_MAX - (as + am), T, &r1, &r2, &r3);
    *fa = r1 + r2 - r3;
    *fm = -r2;
}

/* the zero-rate start of either transformation at T^n (R6, R7, R14).  The
 * alpha_s -> beta start needs D = 0.9 - X_alpha^eq > 0 (Appendix A; R8):
 * below the alpha_s -> beta end temperature X_alpha^eq = 0.9, and a state
 * whose alpha total exceeds it only by rounding is not starting anything. */
static int startup_regime(double as, double am, double bt, double T, double dt)
{
    double xa = as + am, xeq = orc_alpha_eq(T);
    if (xa < xeq && !(as > 0.0)) return 1;
    if (xa > xeq && xeq < X_ALPHA_MAX && (bt > 0.0 ? bt : 0.0) * dt <= STARTUP_LIMIT) return 1;
    return 0;
}

/* One Crank-Nicolson step of the diffusive term followed by g at T^{n+1},
 * the nonlinear equation solved by fixed-point iteration.  Returns the number
 * of iterations taken (0 for a start-up step), negated when the WRMS norm of
 * the residual did not fall below 1 within max_iter iterations. */
int orc_step_cn(double *as_, double *am_, double *b_, double *bt_, double Tn, double Tn1, double dt,
                int max_iter, double eps_abs, double eps_rel)
{
    const double as = *as_, am = *am_;
    if (startup_regime(as, am, *bt_, Tn, dt)) {
        /* the implicit scheme corrects at T^{n+1} (eq. implicit_correction) */
        step_at(as_, am_, b_, bt_, Tn, Tn1, dt);
        return 0;
    }
    double fa_n, fm_n;
    diff_rates(as, am, Tn, &fa_n, &fm_n);
    /* initial iterate: the correction at T^{n+1} applied to m^n (R12) */
    double a = as, m = am;
    double b = orc_correct(Tn1, &a, &m);
    double fa, fm;
    diff_rates(a, m, Tn1, &fa, &fm);
    int it = 0, converged = 0;
    while (it < max_iter) {
        double a1 = as + 0.5 * dt * (fa + fa_n);
        double m1 = am + 0.5 * dt * (fm + fm_n);
        b = orc_correct(Tn1, &a1, &m1);
        double fa1, fm1;
        diff_rates(a1, m1, Tn1, &fa1, &fm1);
        /* residual of the implicit equation at the new iterate */
        double ra = 0.5 * dt * (fa1 - fa), rm = 0.5 * dt * (fm1 - fm);
        double wa = 1.0 / (eps_abs + fabs(a1) * eps_rel), wm = 1.0 / (eps_abs + fabs(m1) * eps_rel);
        double e = 0.5 * ((ra * wa) * (ra * wa) + (rm * wm) * (rm * wm));
        a = a1;
        m = m1;
        fa = fa1;
        fm = fm1;
        ++it;
        if (e < 1.0) {
            converged = 1;
            break;
        }
    }
    *as_ = a;
    *am_ = m;
    *b_ = b;
    *bt_ = X_ALPHA_MAX - (a + m);
    return converged ? it : -it;
}

/* number of equal substeps of a step of length dt (R15) */
int64_t orc_substeps(double dt, double dt_sub)
{
    if (!(dt > dt_sub)) return 1;
    return (int64_t)ceil(dt / dt_sub * (1.0 - 1e-12));
}

/* implicit step with subcycling for n points; returns the number of
 * substeps (over all points) whose iteration hit max_iter; iters (may be
 * NULL) receives each point's total iteration count */
int64_t orc_step_implicit_n(int64_t n, double *as, double *am, double *b, double *bt, const double *Tn,
                            const double *Tn1, double dt, double dt_sub, int max_iter, double eps_abs,
                            double eps_rel, int64_t *iters)
{
    int64_t bad = 0;
    const int64_t ns = orc_substeps(dt, dt_sub);
    const double h = dt / (double)ns;
    for (int64_t i = 0; i < n; ++i) {
        int64_t total = 0;
        for (int64_t s = 0; s < ns; ++s) {
            double T0 = Tn[i] + (Tn1[i] - Tn[i]) * (double)s / (double)ns;
            double T1 = Tn[i] + (Tn1[i] - Tn[i]) * (double)(s + 1) / (double)ns;
            int it = orc_step_cn(&as[i], &am[i], &b[i], &bt[i], T0, T1, h, max_iter, eps_abs, eps_rel);
            if (it < 0) {
                ++bad;
                it = -it;
            }
            total += it;
        }
        if (iters) iters[i] = total;
    }
    return bad;
}

/* ---------------- temperature model (reading R9) ----------------
 *
 * Point source of absorbed power q moving at speed v along a straight track
 * on the adiabatic surface of a semi-infinite body, switched on at t_on:
 * time integral of instantaneous point sources (image factor 2),
 *
 *   F = q/(4 pi k R) [ e^{-v(xi+R)/(2 alpha)} erfc((R - v tau)/s)
 *                    + e^{-|x-P0|^2/(4 alpha tau)} erfcx((R + v tau)/s) ],
 *
 * tau = t - t_on, s = 2 sqrt(alpha tau), xi the coordinate along the motion
 * relative to the current source position, R the distance to it.  A track
 * switched off after dur contributes F(P0, tau) - F(P1, tau - dur), with P1
 * its end point (a virtual source continuing from P1 cancels the rest).
 * T = min(T_clamp, T0 + sum over the last `window` tracks switched on by t).
 */

#define R_EPS 1e-9 /* [m]: closer than this to a switched-on source the clamp applies */
#define R_OFF 5e-7 /* [m]: see reading R16 */

/* erfcx(y) = exp(y^2) erfc(y) for y >= 0: direct product below 25, above it
 * the asymptotic series of Abramowitz & Stegun 7.1.23. */
double orc_erfcx(double y)
{
    if (y < 25.0) return exp(y * y) * erfc(y);
    double t = 1.0 / (2.0 * y * y), term = 1.0, sum = 1.0;
    for (int k = 1; k <= 10; ++k) {
        term *= -(2.0 * k - 1.0) * t;
        sum += term;
    }
    return sum / (y * sqrt(M_PI));
}

/* one switched-on source that started at (x0, y0, z0) tau ago; R precomputed */
static double source_F(double x0, double y0, double z0, double ux, double uy,
                       double q, double v, double tau, double k, double alpha,
                       double x, double y, double z)
{
    double xs = x0 + v * tau * ux, ys = y0 + v * tau * uy;
    double dx = x - xs, dy = y - ys, dz = z - z0;
    double R = sqrt(dx * dx + dy * dy + dz * dz);
    double xi = dx * ux + dy * uy;
    double s = 2.0 * sqrt(alpha * tau);
    double e0x = x - x0, e0y = y - y0;
    double d02 = e0x * e0x + e0y * e0y + dz * dz;
    double t1 = exp(-v * (xi + R) / (2.0 * alpha)) * erfc((R - v * tau) / s);
    double t2 = exp(-d02 / (4.0 * alpha * tau)) * orc_erfcx((R + v * tau) / s);
    return q / (4.0 * M_PI * k * R) * (t1 + t2);
}

double orc_source_F(const double *tr, double tau, double k, double alpha,
                    double x, double y, double z)
{
    return source_F(tr[0], tr[1], tr[2], tr[3], tr[4], tr[7], tr[8], tau, k, alpha, x, y, z);
}

/* index of the last track switched on by time t, or -1 (tracks sorted by
 * t_on).  A track counts as switched on when t_on <= t + 1e-12 s, so that the
 * same window results whether a time is formed as t0 + n dt or as (s + n) dt
 * (the two can differ by an ulp exactly where a track starts). */
#define T_ON_TOL 1e-12
static int64_t last_on(const double *tracks, int64_t n_tracks, double t)
{
    int64_t lo = 0, hi = n_tracks; /* first index with t_on > t + tol */
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (tracks[mid * 9 + 5] <= t + T_ON_TOL) lo = mid + 1;
        else hi = mid;
    }
    return lo - 1;
}

/* sp = {k, alpha, T0, T_clamp, window} */
double orc_temperature(const double *tracks, int64_t n_tracks, const double *sp,
                       double x, double y, double z, double t)
{
    double k = sp[0], alpha = sp[1], T0 = sp[2], Tc = sp[3];
    int64_t W = (int64_t)sp[4];
    int64_t c = last_on(tracks, n_tracks, t);
    double T = T0;
    for (int64_t j = c; j >= 0 && j > c - W; --j) {
        const double *tr = tracks + j * 9;
        double tau = t - tr[5];
        if (!(tau > 0.0)) continue;
        double ux = tr[3], uy = tr[4], v = tr[8], dur = tr[6];
        double xs = tr[0] + v * tau * ux, ys = tr[1] + v * tau * uy;
        double dx = x - xs, dy = y - ys, dz = z - tr[2];
        double R = sqrt(dx * dx + dy * dy + dz * dz);
        double px = x, py = y, pz = z;
        if (tau > dur) {
            /* switched off: the current position is virtual and the field is
             * smooth there (the two singular parts cancel exactly); within
             * R_OFF of it the contribution is taken at R_OFF below it (R16) */
            if (R < R_OFF) {
                px = xs;
                py = ys;
                pz = tr[2] - R_OFF;
            }
        } else if (R < R_EPS) {
            return Tc;
        }
        double C = orc_source_F(tr, tau, k, alpha, px, py, pz);
        if (tau > dur) {
            double x1 = tr[0] + v * dur * ux, y1 = tr[1] + v * dur * uy;
            C -= source_F(x1, y1, tr[2], ux, uy, tr[7], v, tau - dur, k, alpha, px, py, pz);
        }
        T += C;
    }
    return T > Tc ? Tc : T;
}

void orc_temperature_n(const double *tracks, int64_t n_tracks, const double *sp,
                       const double *xyz, int64_t n, double t, double *T_out)
{
    for (int64_t i = 0; i < n; ++i)
        T_out[i] = orc_temperature(tracks, n_tracks, sp, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], t);
}

/* Run n_steps explicit steps at the given points with the analytic
 * temperature: t_s = t0 + s*dt; point-major (each point's history in turn).
 * Points with z > z_top + 1e-3 h are inactive and left untouched. */
void orc_scan_run(const double *tracks, int64_t n_tracks, const double *sp,
                  const double *xyz, int64_t n, double z_top, double h,
                  double t0, double dt, int64_t n_steps,
                  double *as, double *am, double *b, double *bt, int n_threads)
{
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads)
#endif
    for (int64_t i = 0; i < n; ++i) {
        double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (!(z <= z_top + 1e-3 * h)) continue;
        double Tn = orc_temperature(tracks, n_tracks, sp, x, y, z, t0);
        for (int64_t s = 0; s < n_steps; ++s) {
            double t1 = t0 + (double)(s + 1) * dt;
            double Tn1 = orc_temperature(tracks, n_tracks, sp, x, y, z, t1);
            orc_step(&as[i], &am[i], &b[i], &bt[i], Tn, Tn1, dt);
            Tn = Tn1;
        }
    }
}

/* the same run with the implicit scheme at every step (Crank-Nicolson,
 * fixed point, the paper's tolerances; steps longer than dt_sub are split
 * with T linear between the analytic end values, R15).  Returns the number
 * of substeps whose iteration hit max_iter. */
int64_t orc_scan_run_implicit(const double *tracks, int64_t n_tracks, const double *sp,
                              const double *xyz, int64_t n, double z_top, double h,
                              double t0, double dt, int64_t n_steps, double dt_sub, int max_iter,
                              double *as, double *am, double *b, double *bt, int n_threads)
{
    int64_t bad = 0;
    const int64_t ns = orc_substeps(dt, dt_sub);
    const double hs = dt / (double)ns;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads) reduction(+ : bad)
#endif
    for (int64_t i = 0; i < n; ++i) {
        double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (!(z <= z_top + 1e-3 * h)) continue;
        double Tn = orc_temperature(tracks, n_tracks, sp, x, y, z, t0);
        for (int64_t s = 0; s < n_steps; ++s) {
            double t1 = t0 + (double)(s + 1) * dt;
            double Tn1 = orc_temperature(tracks, n_tracks, sp, x, y, z, t1);
            for (int64_t k = 0; k < ns; ++k) {
                double Ta = Tn + (Tn1 - Tn) * (double)k / (double)ns;
                double Tb = Tn + (Tn1 - Tn) * (double)(k + 1) / (double)ns;
                if (orc_step_cn(&as[i], &am[i], &b[i], &bt[i], Ta, Tb, hs, max_iter, 1e-10, 1e-3) < 0) ++bad;
            }
            Tn = Tn1;
        }
    }
    return bad;
}

/* same, with the temperature history given per point (n x (n_steps+1)) */
void orc_history_run(int64_t n, int64_t n_steps, const double *T_hist, double dt,
                     double *as, double *am, double *b, double *bt)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t s = 0; s < n_steps; ++s)
            orc_step(&as[i], &am[i], &b[i], &bt[i], T_hist[i * (n_steps + 1) + s],
                     T_hist[i * (n_steps + 1) + s + 1], dt);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
