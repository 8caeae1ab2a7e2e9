/*
 * mstruct: MI355X (gfx950) library for the pointwise phase update of the
 * Ti-6Al-4V microstructure model of Proell et al., "A highly efficient
 * computational approach for part-scale microstructure predictions in
 * Ti-6Al-4V additive manufacturing" (arXiv 2402.17580).
 *
 * Conventions for every entry point
 *  - Return value: MSTRUCT_OK (0) or a negative mstruct_status.  Nothing
 *    throws across this boundary and nothing calls exit().
 *  - Argument checks happen on the host before anything is enqueued; a
 *    rejected call enqueues no work and leaves every buffer untouched.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream)
 *    and runs asynchronously; device-side faults surface as MSTRUCT_EDEVICE
 *    at the next call that synchronises.  A context must not be used by two
 *    host threads at the same time, and its calls must be ordered (one
 *    stream, or ordering enforced by the caller).
 *  - Per-point arrays are device pointers owned by the caller (float32,
 *    structure of arrays, n entries).  The library never frees them and keeps
 *    no pointer to them after a call returns.  The context owns only small
 *    buffers of its own (scan tables, counters, network weights).
 *  - Units: temperature K, time s, length m, power W.
 */
#ifndef MSTRUCT_H
#define MSTRUCT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MSTRUCT_OK = 0,
    MSTRUCT_EINVAL = -1,       /* invalid argument (null, size, non-finite, range) */
    MSTRUCT_EDEVICE = -2,      /* HIP runtime error (see mstruct_last_error) */
    MSTRUCT_ENOMEM = -3,       /* context could not allocate its own buffers */
    MSTRUCT_EUNSUPPORTED = -4, /* option not available (e.g. window > 4) */
    MSTRUCT_ESTATE = -5        /* context not ready (e.g. surrogate without weights) */
} mstruct_status;

typedef struct mstruct_ctx mstruct_ctx;

/* Phase fractions of n points, device float32 arrays (structure of arrays).
 *
 * xbt is optional (NULL: not used): a device float64 array of n values that
 * carries the shifted beta fraction X~beta = 0.9 - X_alpha of points whose
 * alpha_s -> beta transformation is starting.  Its early values are far below
 * the float32 resolution of X_beta = 0.1 + X~beta (e.g. 1e-80 after one
 * microsecond at 1200 K), which is why the paper keeps X~beta apart
 * (Appendix A); without xbt the float32 state cannot leave that start within
 * holds of seconds at 935-1273 K.  A point is tracked while it has no
 * martensite, dissolves at T^n (X_alpha > X_alpha^eq) and X~beta < 2^-12;
 * above that alpha_s itself resolves X~beta.  NaN marks "not tracked": fill
 * the array with NaN before its first use.  mstruct_step, mstruct_step_implicit
 * and fused PLAIN and IMPLICIT modes read and write it (8 more bytes per
 * point each way); fused SURROGATE mode rejects it (MSTRUCT_EUNSUPPORTED).
 * A value that disagrees with the fractions (martensite present, or alpha_s
 * not 0.9 - X~beta to float32 rounding) is ignored; after the fractions are
 * changed by other means (the surrogate, mstruct_correct, the caller) fill
 * it with NaN again. */
typedef struct {
    float *beta;    /* X_beta */
    float *alpha_s; /* X_alpha_s (stable alpha) */
    float *alpha_m; /* X_alpha_m (martensite) */
    int64_t n;
    double *xbt;    /* optional tracked X~beta, see above */
} mstruct_phases;

/* Laser scan as a host table of straight tracks (row-major n_tracks x 9,
 * float64, sorted by t_on): x0, y0, z0, ux, uy, t_on, dur, q, v  -- start
 * point on the layer surface [m], in-plane unit direction, switch-on time
 * [s], on-duration [s], absorbed power [W], speed [m/s].  The temperature at
 * a point is T0 plus the superposed contributions of the last `window` tracks
 * switched on by time t, i.e. with t_on <= t + 1e-12 s (each a moving point
 * source on the adiabatic surface
 * of a semi-infinite body, switched on at t_on and off after dur), clamped at
 * T_clamp.  window is 1..4. */
typedef struct {
    const double *tracks;
    int64_t n_tracks;
    double conductivity; /* k [W/(m K)] */
    double diffusivity;  /* alpha [m^2/s] */
    double T0;           /* far-field / initial temperature [K] */
    double T_clamp;      /* upper clamp [K] */
    int window;
} mstruct_scan;

/* Material points on a regular box grid: point (i, j, k) sits at
 * (ox + i h, oy + j h, oz - k h) with box linear index i + nx (j + ny k).
 * `index` (device int32, n distinct box linear indices, each in
 * [0, nx*ny*nz), in any order; not checked on the device) selects a masked
 * subset.  The fused kernels take 64 consecutive entries per wave, so an
 * order that keeps each 64 close together in a plane lets more waves skip
 * launches (see MSTRUCT_OPTION_SKIP_COLD_WAVES): e.g. each plane's points
 * through its 8 x 8 tiles, row by row (a sorted list gives parts of rows,
 * which only suit tracks along x);
 * NULL means all nx*ny*nz box points in linear order (then n must equal
 * nx*ny*nz).  Points with z > z_top + 1e-3 h are inactive: the fused call
 * leaves them untouched (material not yet deposited). */
typedef struct {
    int64_t nx, ny, nz;
    double h, ox, oy, oz;
    const int32_t *index;
    int64_t n;
    double z_top;
} mstruct_points;

enum { MSTRUCT_MODE_PLAIN = 0, MSTRUCT_MODE_SURROGATE = 1, MSTRUCT_MODE_IMPLICIT = 2 };

/* Float64 state for mstruct_step_f64 (device arrays of n points, caller-owned). */
typedef struct {
    double *beta;
    double *alpha_s;
    double *alpha_m;
    int64_t n;
} mstruct_phases_f64;

/* exp2 / log2 used by mstruct_step_f64 */
enum { MSTRUCT_F64_LIBRARY = 0, MSTRUCT_F64_SYNTH = 1, MSTRUCT_F64_PAPER = 2 };

/* Model parameters of a context: the constants of Table 1 (thermal), Table 2
 * (phase-transformation temperatures and equilibrium laws) and Table 3
 * (diffusion laws) of the paper with the regularisation width T_as,reg =
 * 100 K (Sec. 2.2), and the two readings of the paper that can be switched:
 *  - correction_T: the temperature at which the explicit scheme applies the
 *    correction g -- T^{n+1} as eq. explicit_correction writes it
 *    (MSTRUCT_CORRECTION_T_NEXT, default) or the T^n that Algorithm 2 passes
 *    (MSTRUCT_CORRECTION_T_PREV).  The implicit scheme corrects at T^{n+1}
 *    either way (eq. implicit_correction).
 *  - martensite_mode: below the martensite start, eq.
 *    inst_martensite_formation raises alpha_m to the pseudo-equilibrium of
 *    eq. equilibrium_phase_am and never lowers it (MSTRUCT_MARTENSITE_MAX,
 *    default; reheating below the start keeps martensite, whose dissolution
 *    has its own law), or sets it to that value literally
 *    (MSTRUCT_MARTENSITE_ASSIGN), lowering it on reheating.
 * The constants are compiled into the kernels as immediate operands:
 * mstruct_init accepts only their values from mstruct_default_params
 * (MSTRUCT_EUNSUPPORTED otherwise; other values need a rebuild).  Fused
 * SURROGATE mode needs the default readings (its network was trained on
 * them). */
typedef struct {
    double T_solidus, T_liquidus, T_ambient;                /* Table 1 [K] */
    double T_alpha_s_start, T_alpha_s_end, T_alpha_m_start; /* Table 2 [K] */
    double k_alpha_eq, k_alpha_m_eq;                        /* Table 2 [1/K] */
    double c_alpha_s, c_beta, k1, k2, k3, f;                /* Table 3: k1 [1/s], k2 [K], k3 [1/K] */
    double T_alpha_s_reg;                                   /* [K] */
    int correction_T;
    int martensite_mode;
} mstruct_params;

enum { MSTRUCT_CORRECTION_T_NEXT = 0, MSTRUCT_CORRECTION_T_PREV = 1 };
enum { MSTRUCT_MARTENSITE_MAX = 0, MSTRUCT_MARTENSITE_ASSIGN = 1 };

/* Fill *p with the paper's values and the default readings. */
int mstruct_default_params(mstruct_params *p);

/* Create a context on HIP device `device` with the given parameters (NULL:
 * mstruct_default_params); the caller's current device is restored.  *out
 * receives the context; free it with mstruct_destroy.  Also takes, once per
 * device, the address of the device array of
 * mstruct_fused_scan_steps_noalloc. */
int mstruct_init(const mstruct_params *params, int device, mstruct_ctx **out);
int mstruct_destroy(mstruct_ctx *ctx);
const char *mstruct_status_string(int status);
/* Last error message recorded on ctx (never NULL). */
const char *mstruct_last_error(const mstruct_ctx *ctx);

/* One explicit time step for all n points, in place: Sec. 3.1 of the paper,
 * eq. explicit_integration (forward Euler on the diffusive rates, eqs.
 * beta_to_alpha_s, alpha_m_to_alpha_s, alpha_s_to_beta, at T_prev) followed
 * by eq. explicit_correction (instantaneous martensite formation and
 * dissolution, alpha_s regularisation, continuity constraints, at T_next),
 * with the closed-form start of diffusion from zero-rate states (Sec. 3.1,
 * Appendix A).  This is the local update of Algorithm 1 / Algorithm 2.
 * T_prev, T_next: device float32 [n] temperatures at t_n and t_n + dt.  The
 * input beta is not read (X_beta follows from the sum rule, eq.
 * time_integration_beta_postprocess); alpha_s, alpha_m are read, all three
 * are written.  dt > 0 and finite.  Arrays need no particular alignment
 * (16-byte alignment of all five enables vector access). */
int mstruct_step(mstruct_ctx *ctx, const float *T_prev, const float *T_next, double dt,
                 const mstruct_phases *ph, void *stream);

/* The explicit step of mstruct_step (Algorithm 1 with Algorithm 2) in
 * float64 for n points, in place: T_prev, T_next and the three fractions are
 * device float64 arrays (40 bytes read and 24 written per point).  math
 * MSTRUCT_F64_LIBRARY uses the device math library's exp2, log2 and expm1;
 * MSTRUCT_F64_SYNTH builds exp2 and log2 from the bit pattern of the double
 * and a short series on the reduced argument (the technique of Sec. 3.3,
 * with series of full double accuracy); both agree with the reference to a
 * few float64 ulps.  MSTRUCT_F64_PAPER uses the paper's own method of Sec.
 * 3.3: eqs. exp_algorithm_1 - exp_algorithm_3 and eq. ln_approx with the
 * correction polynomials of Table tab:coefficients_approx_correction in
 * Estrin's scheme, whose accuracy is that of the fits: 2^y to 1.2e-10
 * relative, log2 to 3.0e-8 absolute.  dt > 0 and finite; asynchronous on
 * the stream. */
int mstruct_step_f64(mstruct_ctx *ctx, const double *T_prev, const double *T_next, double dt,
                     const mstruct_phases_f64 *ph, int math, void *stream);

/* One step of the implicit scheme (Sec. 3.1, eqs. implicit_integration,
 * implicit_correction, implicit_fp_iteration; the implicit algorithm of
 * Sec. 3.2) for n points, in place: Crank-Nicolson on the diffusive rates
 * with the correction g at T^{n+1}, the nonlinear equation solved by
 * fixed-point iteration from g(T^{n+1}, m^n) until the WRMS norm of the
 * residual over (alpha_s, alpha_m), with eps_abs = 1e-10 and eps_rel = 1e-3,
 * falls below 1, or max_iter iterations (1..1000; the paper's scheme is
 * used with 50).  A state in a start-up regime (zero rate of a starting
 * transformation at T^n) takes the explicit step with its Appendix A closed
 * form.  Steps longer than dt_sub (the paper uses 0.01 s) are split into the
 * fewest equal substeps not longer than dt_sub, with T linear in time
 * (dt / dt_sub at most 1e6).  T_prev, T_next, phases: device float32 arrays
 * of ph->n points, no alignment needed.  unconverged (device, may be NULL)
 * is incremented by the number of substeps whose iteration hit max_iter; the
 * caller zeroes it.  Asynchronous on the stream. */
int mstruct_step_implicit(mstruct_ctx *ctx, const float *T_prev, const float *T_next, double dt,
                          double dt_sub, int max_iter, const mstruct_phases *ph,
                          unsigned long long *unconverged, void *stream);

/* Temperature of the active points at time t (the scan model above), written
 * to T_out[n] (device float32; inactive points get T0). */
int mstruct_temperature(mstruct_ctx *ctx, const mstruct_scan *scan, const mstruct_points *pts,
                        double t, float *T_out, void *stream);

/* n_steps explicit steps t0 + s dt -> t0 + (s+1) dt for the active points
 * with the temperature evaluated from the scan inside the kernel, K steps per
 * launch with the phase state held in registers (Sec. 4.1 names this
 * "subcycling on loaded data").  Simulated time and source positions are
 * computed on the host in float64.  mode PLAIN runs the explicit step of
 * mstruct_step at every step (with compensated accumulation of the Euler
 * increments inside a launch).  mode SURROGATE replaces each block of K steps
 * of a point by one explicit step of K dt (rates at the block-start
 * temperature, correction at the block-end temperature) plus the correction
 * to it predicted by the trained network (applied where the one-step
 * increment of alpha_s or alpha_m exceeds 2^-20; below that one step of K dt
 * is taken as it is), except where the error
 * indicator flags the point (temperature window touching the martensite
 * start, beta-transus or melting bands, or a start-up state), which get the
 * K plain steps; requires weights loaded with mstruct_mlp_set_params.
 * mode IMPLICIT runs the implicit step of mstruct_step_implicit at every
 * step (substep limit 0.01 s, T linear in time between the analytic values
 * at the step ends, at most 50 iterations, compensated accumulation of the
 * increments inside a launch); substeps that hit the cap are counted in the
 * context (see mstruct_implicit_unconverged).  In PLAIN and IMPLICIT modes
 * a wave of points at rest that provably stays below 935 K through a launch
 * skips it, and a wave that no source of a launch reaches takes T = T0 at
 * every step without evaluating the source terms, with the same results bit
 * for bit (see MSTRUCT_OPTION_SKIP_COLD_WAVES).
 * K in 1..64.  pts->n must equal ph->n.  Inside a call beta is not read and
 * is written once, by the last launch (it follows from the sum rule). */
int mstruct_fused_scan_steps(mstruct_ctx *ctx, const mstruct_scan *scan, const mstruct_points *pts,
                             double t0, double dt, int64_t n_steps, int K, int mode,
                             const mstruct_phases *ph, void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): mstruct_fused_scan_steps in PLAIN or
 * IMPLICIT mode (SURROGATE: MSTRUCT_EUNSUPPORTED) with the same arguments,
 * kernels and results, bit for bit, that allocates nothing.  Its per-call
 * buffers -- the scan table with the launch envelopes, the waves' boxes and
 * the wave flags -- live in one 32 MiB device array per GPU, which the
 * library holds until the process ends; the table is uploaded from a static
 * host array.  Limit: the table of a call, (n_steps + 1) * window records of
 * 64 bytes plus the envelopes (at most (K + 1) * window records per launch)
 * and 8 bytes per launch, must fit in 4 MiB (65,536 records), else
 * MSTRUCT_EINVAL and nothing is enqueued; wave flags are used when at least
 * one launch of them fits in the remaining 28 MiB (2 bytes per 64 points,
 * plus 24 bytes per 64 points and per 4096 points with an index list),
 * otherwise the call runs without them (same results).  Every call on a GPU uses that GPU's one
 * array: calls on different streams, or from different host threads, that
 * overlap in time race on it; calls on one stream are ordered.  The host
 * part of these calls is serialised by a lock, and each waits until the
 * previous call's table upload has completed. */
int mstruct_fused_scan_steps_noalloc(mstruct_ctx *ctx, const mstruct_scan *scan, const mstruct_points *pts,
                                     double t0, double dt, int64_t n_steps, int K, int mode,
                                     const mstruct_phases *ph, void *stream);

/* Context options (value 0 or 1 unless stated).
 * MSTRUCT_OPTION_SKIP_COLD_WAVES (default 1): before each launch of fused
 * PLAIN or IMPLICIT mode the host lists every track that occupies a window
 * slot at any of the launch's time points, with its positions at the first
 * and last of them.  Each point bounds every track over the whole launch in
 * two ways.  (1) A wave whose points are all at rest (alpha_s = 0.9, no
 * martensite) and whose temperatures provably stay below 935 K, where both
 * schemes leave such a state unchanged, skips the launch: no temperature, no
 * step and no store of alpha_s, alpha_m.  (2) A wave whose points drop every
 * term of every track by the drop test of the temperature model (a term
 * provably below 1e-4 K is dropped) has T = T0 throughout and skips the
 * evaluation of the sources.  Without xbt, each call also bounds the box
 * of every wave of 64 points (of the box, see MSTRUCT_OPTION_TILE_WAVES, or
 * 64 consecutive points of the index list) against
 * every launch's tracks in a pre-pass, and the context remembers which such
 * waves were at rest: from the second launch of a call such a wave reads
 * neither its state nor a track.  For this the context keeps 2 n/64 bytes
 * (and 24 (n/64 + n/4096) bytes of boxes with an index list) plus at most
 * 256 MiB of still flags per call on the device, until mstruct_destroy.  The results are the same bit for bit as with 0, which
 * evaluates every temperature and takes every step (for comparison). */
enum {
    MSTRUCT_OPTION_SKIP_COLD_WAVES = 1,
    MSTRUCT_OPTION_COUNT_WAVES = 2,
    MSTRUCT_OPTION_TILE_WAVES = 3,
    MSTRUCT_OPTION_WAVE_TILE_WIDTH = 4
};
/* MSTRUCT_OPTION_TILE_WAVES (default 1): on a box grid (no index list) the
 * fused kernels may group the points of each plane into waves of a x b = 64
 * points (a along x, a power of two) instead of 64 consecutive points of a
 * row (the "waves" of the option above and of mstruct_wave_counts).  Each
 * call keeps the row order when the tracks on during the call, weighted by
 * their time on, run along x (sum of |uy| at most a tenth of the sum of
 * |ux|) or no track is on, and otherwise takes 8 x 8 tiles (or the nearest
 * of 16 x 4, 4 x 16, 32 x 2, 2 x 32 that divides nx and ny): near the
 * tracks the waves that step then cover fewer points that need not step.
 * With 0, always the row order.  The arrays keep the box order.  PLAIN and IMPLICIT results are
 * the same bit for bit for every shape; in SURROGATE mode, where a wave
 * takes the network only if all its points pass the error indicator, the
 * shape decides where the network acts (both within the surrogate's error).
 * MSTRUCT_OPTION_WAVE_TILE_WIDTH (default 0: chosen per call as above): a
 * power of two a in 1..64 forces tiles of a x (64 / a) points where they
 * divide nx and ny (else the row order); other values MSTRUCT_EINVAL. */
/* MSTRUCT_OPTION_COUNT_WAVES (default 0): fused PLAIN and IMPLICIT launches
 * count, per wave of 64 points, what they read and write, into counters of
 * the context read by mstruct_wave_counts (one atomic per wave and class;
 * for measurement, not for timed runs).  Results are unchanged. */
int mstruct_set_option(mstruct_ctx *ctx, int option, int value);

/* The counts of MSTRUCT_OPTION_COUNT_WAVES since the context was created or
 * last reset (reset != 0 zeroes them after reading); synchronises the
 * stream.  counts[0]: points whose state (alpha_s, alpha_m) a launch read;
 * [1]: points whose state it wrote; waves that read their state and then
 * [2]: were still by the launch certificates (no step, no store), [3]: were
 * cold (T = T0 without evaluating the sources), [4]: evaluated the
 * temperature at every step; [5]: waves still by their wave flags, which
 * read nothing.  Beta, written once per call for every active point, is not
 * counted.  Fused PLAIN launches also count the whole sub-blocks of 8 steps
 * of the waves of [4] ([6]) and those of them in which every point passes
 * the surrogate's default error indicator (see mstruct_mlp_set_params) at
 * the sub-block's end temperatures ([7]). */
int mstruct_wave_counts(mstruct_ctx *ctx, int64_t counts[8], int reset, void *stream);

/* Number of substeps of fused IMPLICIT runs on this context whose fixed-point
 * iteration hit the cap, since the context was created or last reset
 * (reset != 0 zeroes it after reading).  Synchronises the stream. */
int mstruct_implicit_unconverged(mstruct_ctx *ctx, int64_t *count, int reset, void *stream);

/* dst[i] = src[idx[i]] for i < m (device arrays). */
int mstruct_gather(mstruct_ctx *ctx, const float *src, const int64_t *idx, int64_t m, float *dst,
                   void *stream);

/* Count points violating the model's invariants (fractions outside [0, 1],
 * alpha_s + alpha_m > 0.9 + tol, phase sum differing from X_sol(T) by more
 * than tol when T is given, NaN).  T may be NULL.  Synchronises the stream;
 * *violations receives the count. */
int mstruct_check_invariants(mstruct_ctx *ctx, const mstruct_phases *ph, const float *T, float tol,
                             int64_t *violations, void *stream);

/* The correction g of eq. explicit_correction alone, at temperatures T[n]
 * (device float32), in place: instantaneous martensite formation and
 * dissolution, alpha_s regularisation, continuity constraints; beta written
 * from the sum rule.  Used to separate instantaneous from diffusive changes. */
int mstruct_correct(mstruct_ctx *ctx, const float *T, const mstruct_phases *ph, void *stream);

/* ---- learned surrogate (not part of the paper): MLP 6 -> 64 -> 64 -> 3,
 * ReLU, BF16 MFMA products with float32 accumulation ----
 * Raw inputs per sample: (T_n, T_{n+K}, ln dt, beta, alpha_s, alpha_m), each
 * normalised in the library as (x - in_mean) / in_scale.  Network outputs
 * times out_scale are the differences of (alpha_s, alpha_m, beta) between K
 * explicit steps of dt and one explicit step of K dt over the same block.  Parameter
 * vector (float32, MSTRUCT_MLP_NPARAM entries, row = output unit):
 * W1[64][6], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]. */
#define MSTRUCT_MLP_NPARAM 4803

/* Upload parameters (host float32) and normalisation (host in_mean[6],
 * in_scale[6] > 0, out_scale[3] > 0); indicator (host float32[4] or NULL for
 * the defaults 823, 1398, 1853, 50): the surrogate is used for a K-block only
 * when both block-end temperatures lie below indicator[0] K or both inside
 * [indicator[1], indicator[2]] K, and they differ by at most indicator[3] K.
 * Resets the optimiser state.  Synchronises the device. */
int mstruct_mlp_set_params(mstruct_ctx *ctx, const float *params, const float *in_mean, const float *in_scale,
                           const float *out_scale, const float *indicator);
/* Copy the float32 parameters to a host array (synchronises). */
int mstruct_mlp_get_params(mstruct_ctx *ctx, float *params);

/* Network on B samples: X device float32 [B][6] raw inputs; Y device float32
 * [B][3] = outputs times out_scale. */
int mstruct_mlp_forward(mstruct_ctx *ctx, const float *X, int64_t B, float *Y, void *stream);

/* Loss 0.5/B sum_i ||f(norm(X_i)) - Y_i / out_scale||^2 and its gradient with
 * respect to the parameters (layout above): grad device float32
 * [MSTRUCT_MLP_NPARAM], loss device float32 [1].  Deterministic (per-wave
 * partial sums reduced in a fixed order).  B >= 1. */
int mstruct_mlp_grad(mstruct_ctx *ctx, const float *X, const float *Y, int64_t B, float *grad, float *loss,
                     void *stream);

/* One Adam step (betas 0.9, 0.999, eps 1e-8, learning rate lr) on the
 * context's parameters with the gradient of the batch; loss (device float32
 * [1], may be NULL) receives the batch loss before the step. */
int mstruct_mlp_train_step(mstruct_ctx *ctx, const float *X, const float *Y, int64_t B, float lr, float *loss,
                           void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MSTRUCT_H */
