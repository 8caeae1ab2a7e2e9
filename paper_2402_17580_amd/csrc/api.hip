// C-ABI of the mstruct library: argument checks, the context, float64
// bookkeeping of simulated time and source positions, and kernel launches.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "../../include/mstruct.h"
#include "kernels.h"
#include "mlp.h"

using namespace mstruct;

namespace {

constexpr int kSlots = 4;  // tables in flight per context

// set-up of the allocation-free fused call's device array (see below)
int scratch_setup(int device);

struct TableSlot {
    SrcRec* host = nullptr;  // pinned staging
    SrcRec* dev = nullptr;
    size_t cap = 0;  // records
    hipEvent_t done = nullptr;
    bool pending = false;
};

}  // namespace

struct mstruct_ctx {
    int device = 0;
    std::string err;
    TableSlot slots[kSlots];
    int next_slot = 0;
    unsigned long long* counter = nullptr;
    unsigned long long* implicit_bad = nullptr;  // substeps of fused implicit runs that hit the cap
    unsigned long long* stats = nullptr;         // wave counts of fused launches (kStatCount)
    bool count_waves = false;                    // MSTRUCT_OPTION_COUNT_WAVES
    bool skip_cold = true;                       // MSTRUCT_OPTION_SKIP_COLD_WAVES
    bool tile_waves = true;                      // MSTRUCT_OPTION_TILE_WAVES
    int tile_width = 0;                          // MSTRUCT_OPTION_WAVE_TILE_WIDTH (0: chosen per call)
    Readings rd{false, false};                   // mstruct_params' correction_T and martensite_mode
    // per-wave flags of fused calls on box grids: rest flags, then the still
    // flags of a chunk of launches
    uint8_t* wave_flags = nullptr;
    size_t wave_flags_cap = 0;
    // the box of each wave of a call on an index list
    GridBox* wave_boxes = nullptr;
    size_t wave_boxes_cap = 0;
    MlpState mlp;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int fail(mstruct_ctx* ctx, int code, const char* fmt, const char* detail = "") {
    if (ctx) {
        char buf[512];
        snprintf(buf, sizeof buf, fmt, detail);
        ctx->err = buf;
    }
    return code;
}

int hip_fail(mstruct_ctx* ctx, hipError_t e, const char* where) {
    if (ctx) ctx->err = std::string(where) + ": " + hipGetErrorString(e);
    return MSTRUCT_EDEVICE;
}

#define HIP_CHECK(ctx, expr)                                   \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

int check_phases(mstruct_ctx* ctx, const mstruct_phases* ph) {
    if (!ph) return fail(ctx, MSTRUCT_EINVAL, "phases is NULL");
    if (ph->n < 0) return fail(ctx, MSTRUCT_EINVAL, "phases n < 0");
    if (ph->n > 0 && (!ph->beta || !ph->alpha_s || !ph->alpha_m))
        return fail(ctx, MSTRUCT_EINVAL, "phase array is NULL");
    if (ph->n >= (int64_t)1 << 31) return fail(ctx, MSTRUCT_EINVAL, "more than 2^31 - 1 points");
    return MSTRUCT_OK;
}

int check_scan(mstruct_ctx* ctx, const mstruct_scan* sc) {
    if (!sc) return fail(ctx, MSTRUCT_EINVAL, "scan is NULL");
    if (sc->n_tracks < 0 || (sc->n_tracks > 0 && !sc->tracks)) return fail(ctx, MSTRUCT_EINVAL, "bad track table");
    if (sc->window < 1 || sc->window > 4) return fail(ctx, MSTRUCT_EUNSUPPORTED, "window must be 1..4");
    if (!finite_pos(sc->conductivity) || !finite_pos(sc->diffusivity) || !isfinite(sc->T0) ||
        !isfinite(sc->T_clamp) || sc->T_clamp < sc->T0)
        return fail(ctx, MSTRUCT_EINVAL, "bad scan material constants");
    for (int64_t j = 0; j < sc->n_tracks; ++j) {
        const double* r = sc->tracks + 9 * j;
        for (int c = 0; c < 9; ++c)
            if (!isfinite(r[c])) return fail(ctx, MSTRUCT_EINVAL, "non-finite entry in track table");
        if (!(r[6] >= 0.0) || !(r[7] >= 0.0) || !(r[8] >= 0.0))
            return fail(ctx, MSTRUCT_EINVAL, "track with negative duration, power or speed");
        if (fabs(hypot(r[3], r[4]) - 1.0) > 1e-6) return fail(ctx, MSTRUCT_EINVAL, "track direction not unit");
        if (j > 0 && r[5] < r[5 - 9]) return fail(ctx, MSTRUCT_EINVAL, "tracks not sorted by t_on");
    }
    return MSTRUCT_OK;
}

// smallest plane k with oz - k h <= z_top + 1e-3 h (nz if none)
int64_t first_active_plane(const mstruct_points* p) {
    for (int64_t k = 0; k < p->nz; ++k)
        if (p->oz - (double)k * p->h <= p->z_top + 1e-3 * p->h) return k;
    return p->nz;
}

int make_geom(mstruct_ctx* ctx, const mstruct_points* p, int64_t n, PointGeom& pg) {
    if (!p) return fail(ctx, MSTRUCT_EINVAL, "points is NULL");
    const int64_t lim = (int64_t)1 << 31;  // each factor below 2^31 first, so no product overflows
    if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0 || p->nx >= lim || p->ny >= lim || p->nz >= lim ||
        p->nx * p->ny >= lim || p->nx * p->ny * p->nz >= lim)
        return fail(ctx, MSTRUCT_EINVAL, "bad box dimensions (at most 2^31 - 1 points)");
    if (!finite_pos(p->h) || !isfinite(p->ox) || !isfinite(p->oy) || !isfinite(p->oz) || isnan(p->z_top))
        return fail(ctx, MSTRUCT_EINVAL, "bad grid geometry");
    if (p->n != n) return fail(ctx, MSTRUCT_EINVAL, "points n differs from phases n");
    const int64_t nbox = p->nx * p->ny * p->nz;
    if (!p->index && n != nbox) return fail(ctx, MSTRUCT_EINVAL, "without an index list n must be nx*ny*nz");
    if (p->index && n > nbox) return fail(ctx, MSTRUCT_EINVAL, "index list longer than the box");
    const int64_t k0 = first_active_plane(p);
    pg.index = p->index;
    pg.nx = (int32_t)p->nx;
    pg.nxy = (int32_t)(p->nx * p->ny);
    divide_magic(pg.nx, pg.mag_nx, pg.sh_nx);
    divide_magic(pg.nxy, pg.mag_nxy, pg.sh_nxy);
    pg.k0 = (int32_t)k0;
    pg.tiled = 0;  // row order; see choose_wave_shape
    pg.tw_log = 6;
    pg.tr = 0;
    pg.mag_tr = 0;
    pg.sh_tr = -1;
    pg.r2min = (float)((1e-9 / p->h) * (1e-9 / p->h));
    pg.roff = (float)(5e-7 / p->h);
    if (p->index) {
        pg.first = 0;
        pg.count = n;
    } else {
        pg.first = k0 * p->nx * p->ny;
        pg.count = n - pg.first;
    }
    return MSTRUCT_OK;
}

// The wave shape of a fused call on a box grid: tiles of a x b = 64 points
// of a plane (a = 2^s along x; a = 64 is the row order).  Near the tracks
// the waves that step cover a patch around the current track and the last
// hatches, long along the tracks.  Rows cover it best when the tracks run
// along x (multi-layer block: 57 ms per run against 59 ms with 8 x 8
// tiles); at other angles square tiles do (island block, a seeded rotation
// per layer: 0.60 s against 0.81 s in rows, 0.63-0.76 s with 16 x 4, 4 x 16,
// 32 x 2 or 2 x 32).  So a call takes the row order when its tracks,
// weighted by their time on in [t0, t1], run along x (sum of |uy| at most
// a tenth of the sum of |ux|) or none is on, and otherwise 8 x 8 tiles, or
// the nearest shape that divides the plane.  A forced width
// (MSTRUCT_OPTION_WAVE_TILE_WIDTH) is taken where it divides the plane.
int64_t last_on(const mstruct_scan* sc, double t);
void choose_wave_shape(const mstruct_ctx* ctx, const mstruct_scan* sc, const mstruct_points* p, double t0, double t1,
                       PointGeom& pg) {
    if (!ctx->tile_waves || p->index) return;
    auto fits = [&](int s) { return p->nx % ((int64_t)1 << s) == 0 && p->ny % ((int64_t)1 << (6 - s)) == 0; };
    int best = 6;
    if (ctx->tile_width > 0) {
        int s = 0;
        while ((1 << s) < ctx->tile_width) ++s;
        if (fits(s)) best = s;
    } else {
        double wx = 0.0, wy = 0.0;  // time-weighted |ux|, |uy|
        const int64_t j1 = last_on(sc, t1);
        for (int64_t j = j1; j >= 0; --j) {
            const double* tr = sc->tracks + 9 * j;
            if (tr[5] + tr[6] < t0) break;  // where tracks follow one another, all earlier ones ended too
            const double on = fmin(tr[5] + tr[6], t1) - fmax(tr[5], t0);
            if (!(on > 0.0)) continue;
            wx += on * fabs(tr[3]);
            wy += on * fabs(tr[4]);
        }
        if (wy > 0.1 * wx) {
            for (int s : {3, 4, 2, 5, 1})
                if (fits(s)) {
                    best = s;
                    break;
                }
        }
    }
    if (best == 6) return;
    pg.tiled = 1;
    pg.tw_log = best;
    pg.tr = (int32_t)(p->nx >> best);
    divide_magic(pg.tr, pg.mag_tr, pg.sh_tr);
}

// index of the last track switched on by time t, or -1; a track is on when
// t_on <= t + 1e-12 s, so that t0 + n dt and (s + n) dt (which may differ by
// an ulp where a track starts) give the same window
int64_t last_on(const mstruct_scan* sc, double t) {
    const double tol = 1e-12;
    int64_t lo = 0, hi = sc->n_tracks;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (sc->tracks[9 * mid + 5] <= t + tol) lo = mid + 1;
        else hi = mid;
    }
    return lo - 1;
}

// fewest equal substeps of a step dt that are not longer than dt_sub
int substeps(double dt, double dt_sub) { return dt > dt_sub ? (int)ceil(dt / dt_sub * (1.0 - 1e-12)) : 1; }

// substep limit and iteration cap of the implicit scheme in the fused path (Sec. 3.1)
constexpr double kImplicitDtSub = 0.01;
constexpr int kImplicitMaxIter = 50;

// bytes of still flags per chunk of launches of a fused call
constexpr int64_t kWaveFlagBudget = (int64_t)256 << 20;

void split(double g, int32_t& i, float& f) {
    const double fl = floor(g);
    i = (int32_t)fl;
    f = (float)(g - fl);
}

// window slot w at time t: float64 position and timing -> float32 record
void fill_record(SrcRec& r, const mstruct_scan* sc, const mstruct_points* p, int64_t j, double t) {
    memset(&r, 0, sizeof r);
    r.lamp = -INFINITY;  // unused slot
    if (j < 0) return;
    const double* tr = sc->tracks + 9 * j;
    const double tau = t - tr[5];
    if (!(tau > 0.0) || !(tr[7] > 0.0)) return;
    const double ux = tr[3], uy = tr[4], q = tr[7], v = tr[8], dur = tr[6];
    const double h = p->h, a = sc->diffusivity, k = sc->conductivity;
    const double LOG2E = 1.4426950408889634;
    split((tr[0] + v * tau * ux - p->ox) / h, r.ix, r.fx);
    split((tr[1] + v * tau * uy - p->oy) / h, r.iy, r.fy);
    split((tr[2] - p->oz) / h, r.iz, r.fz);
    r.ux = (float)ux;
    r.uy = (float)uy;
    r.lamp = (float)log2(q / (4.0 * M_PI * k * h));
    r.c1 = (float)(v * h / (2.0 * a) * LOG2E);
    r.vt = (float)(v * tau / h);
    r.is = (float)(h / (2.0 * sqrt(a * tau)));
    r.e2 = (float)(h * h / (4.0 * a * tau) * LOG2E);
    if (tau > dur) {
        const double t1 = tau - dur;
        r.vt1 = (float)(v * t1 / h);
        r.is1 = (float)(h / (2.0 * sqrt(a * t1)));
        r.e21 = (float)(h * h / (4.0 * a * t1) * LOG2E);
    }
}

// build (n_times x W) records for t = t0 + s dt, s = 0..n_times-1
void build_table(SrcRec* out, const mstruct_scan* sc, const mstruct_points* p, double t0, double dt,
                 int64_t n_times) {
    const int W = sc->window;
    for (int64_t s = 0; s < n_times; ++s) {
        const double t = t0 + (double)s * dt;
        const int64_t c = last_on(sc, t);
        for (int w = 0; w < W; ++w) fill_record(out[s * W + w], sc, p, c - w, t);
    }
}

// the most distinct tracks one launch can see: K + 1 time points with W
// window slots each (several tracks may switch on within one step)
constexpr int kMaxLaunchTracks = (64 + 1) * 4;

// Per launch of K steps (time points s0 .. s0 + Kb of the call's table), one
// EnvRec for every track that occupies a window slot at any of them: its
// positions at the first and last of those time points and the constants of
// the last.  env[fc[2 i] .. fc[2 i] + fc[2 i + 1]) belongs to launch i.
// Returns the number of records written, or -1 if more than cap would be
// needed (at most n_launches (K + 1) W are).
int64_t build_envelopes(EnvRec* env, int64_t cap, int32_t* fc, const SrcRec* recs, const mstruct_scan* sc,
                        double t0, double dt, int64_t n_steps, int K) {
    const int W = sc->window;
    int64_t total = 0;
    int64_t ids[kMaxLaunchTracks], lo[kMaxLaunchTracks], hi[kMaxLaunchTracks];
    int64_t li = 0;
    for (int64_t s0 = 0; s0 < n_steps; s0 += K, ++li) {
        const int64_t Kb = (n_steps - s0) < K ? (n_steps - s0) : K;
        int n = 0;  // each (time point, slot) adds at most one track: n <= (Kb + 1) W
        for (int64_t s = s0; s <= s0 + Kb; ++s) {
            const int64_t c = last_on(sc, t0 + (double)s * dt);
            for (int w = 0; w < W; ++w) {
                if (!(recs[s * W + w].lamp > -1e30f)) continue;
                const int64_t j = c - w;
                int k = 0;
                while (k < n && ids[k] != j) ++k;
                if (k == n) {
                    ids[n] = j;
                    lo[n] = s * W + w;
                    hi[n] = s * W + w;
                    ++n;
                } else {
                    hi[k] = s * W + w;
                }
            }
        }
        if (total + n > cap) return -1;
        fc[2 * li] = (int32_t)total;
        fc[2 * li + 1] = n;
        for (int k = 0; k < n; ++k) {
            const SrcRec& a = recs[lo[k]];
            const SrcRec& b = recs[hi[k]];
            EnvRec& e = env[total++];
            memset(&e, 0, sizeof e);
            e.px = (float)((double)b.ix + (double)b.fx);
            e.py = (float)((double)b.iy + (double)b.fy);
            e.pz = (float)((double)b.iz + (double)b.fz);
            e.qx = (float)((double)a.ix + (double)a.fx);
            e.qy = (float)((double)a.iy + (double)a.fy);
            e.ux = b.ux;
            e.uy = b.uy;
            e.lamp = b.lamp;
            e.c1 = b.c1;
            e.e2 = b.e2;
            e.vt = b.vt;
            e.is = b.is;
            if (b.is1 > 0.0f) {
                e.e21 = b.e21;
                e.vt1 = b.vt1;
            }
        }
    }
    return total;
}

// acquire a table slot with room for `records` entries; waits until its
// previous use on the GPU is complete
int acquire_slot(mstruct_ctx* ctx, size_t records, TableSlot*& out) {
    TableSlot& s = ctx->slots[ctx->next_slot];
    ctx->next_slot = (ctx->next_slot + 1) % kSlots;
    if (!s.done) HIP_CHECK(ctx, hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
    if (s.pending) {
        HIP_CHECK(ctx, hipEventSynchronize(s.done));
        s.pending = false;
    }
    if (s.cap < records) {
        if (s.host) HIP_CHECK(ctx, hipHostFree(s.host));
        if (s.dev) HIP_CHECK(ctx, hipFree(s.dev));
        s.host = nullptr;
        s.dev = nullptr;
        s.cap = 0;
        size_t cap = records < 1024 ? 1024 : records + records / 4;
        if (hipHostMalloc((void**)&s.host, cap * sizeof(SrcRec), hipHostMallocDefault) != hipSuccess)
            return fail(ctx, MSTRUCT_ENOMEM, "pinned table allocation failed");
        if (hipMalloc((void**)&s.dev, cap * sizeof(SrcRec)) != hipSuccess)
            return fail(ctx, MSTRUCT_ENOMEM, "device table allocation failed");
        s.cap = cap;
    }
    out = &s;
    return MSTRUCT_OK;
}

int release_slot(mstruct_ctx* ctx, TableSlot* s, hipStream_t st) {
    HIP_CHECK(ctx, hipEventRecord(s->done, st));
    s->pending = true;
    return MSTRUCT_OK;
}

}  // namespace

extern "C" {

const char* mstruct_status_string(int status) {
    switch (status) {
        case MSTRUCT_OK: return "ok";
        case MSTRUCT_EINVAL: return "invalid argument";
        case MSTRUCT_EDEVICE: return "HIP device error";
        case MSTRUCT_ENOMEM: return "out of memory";
        case MSTRUCT_EUNSUPPORTED: return "unsupported option";
        case MSTRUCT_ESTATE: return "context not ready";
        default: return "unknown status";
    }
}

const char* mstruct_last_error(const mstruct_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int mstruct_default_params(mstruct_params* p) {
    if (!p) return MSTRUCT_EINVAL;
    memset(p, 0, sizeof *p);
    using C = Const<double>;
    p->T_solidus = C::Tsol;
    p->T_liquidus = C::Tliq;
    p->T_ambient = C::Tinf;
    p->T_alpha_s_start = C::TasStart;
    p->T_alpha_s_end = C::TasEnd;
    p->T_alpha_m_start = C::TamStart;
    p->k_alpha_eq = C::KalphaEq;
    p->k_alpha_m_eq = C::KamEq;
    p->c_alpha_s = C::Cas;
    p->c_beta = C::Cbeta;
    p->k1 = C::K1;
    p->k2 = C::K2;
    p->k3 = C::K3;
    p->f = C::F;
    p->T_alpha_s_reg = C::Treg;
    p->correction_T = MSTRUCT_CORRECTION_T_NEXT;
    p->martensite_mode = MSTRUCT_MARTENSITE_MAX;
    return MSTRUCT_OK;
}

int mstruct_init(const mstruct_params* params, int device, mstruct_ctx** out) {
    if (!out) return MSTRUCT_EINVAL;
    *out = nullptr;
    mstruct_params p;
    mstruct_default_params(&p);
    if (params) {
        // the model constants are immediate operands of the kernels
        const double got[] = {params->T_solidus, params->T_liquidus, params->T_ambient, params->T_alpha_s_start,
                              params->T_alpha_s_end, params->T_alpha_m_start, params->k_alpha_eq,
                              params->k_alpha_m_eq, params->c_alpha_s, params->c_beta, params->k1, params->k2,
                              params->k3, params->f, params->T_alpha_s_reg};
        const double want[] = {p.T_solidus, p.T_liquidus, p.T_ambient, p.T_alpha_s_start, p.T_alpha_s_end,
                               p.T_alpha_m_start, p.k_alpha_eq, p.k_alpha_m_eq, p.c_alpha_s, p.c_beta, p.k1, p.k2,
                               p.k3, p.f, p.T_alpha_s_reg};
        for (size_t i = 0; i < sizeof got / sizeof got[0]; ++i)
            if (got[i] != want[i]) return MSTRUCT_EUNSUPPORTED;
        if (params->correction_T != MSTRUCT_CORRECTION_T_NEXT && params->correction_T != MSTRUCT_CORRECTION_T_PREV)
            return MSTRUCT_EINVAL;
        if (params->martensite_mode != MSTRUCT_MARTENSITE_MAX && params->martensite_mode != MSTRUCT_MARTENSITE_ASSIGN)
            return MSTRUCT_EINVAL;
        p.correction_T = params->correction_T;
        p.martensite_mode = params->martensite_mode;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return MSTRUCT_EINVAL;
    mstruct_ctx* ctx = new (std::nothrow) mstruct_ctx();
    if (!ctx) return MSTRUCT_ENOMEM;
    ctx->device = device;
    ctx->rd = Readings{p.correction_T == MSTRUCT_CORRECTION_T_PREV, p.martensite_mode == MSTRUCT_MARTENSITE_ASSIGN};
    DeviceGuard g(device);
    if (hipMalloc((void**)&ctx->counter, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void**)&ctx->implicit_bad, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void**)&ctx->stats, kStatCount * sizeof(unsigned long long)) != hipSuccess) {
        if (ctx->counter) (void)hipFree(ctx->counter);
        if (ctx->implicit_bad) (void)hipFree(ctx->implicit_bad);
    if (ctx->stats) (void)hipFree(ctx->stats);
        delete ctx;
        return MSTRUCT_ENOMEM;
    }
    const unsigned long long zero[kStatCount] = {};
    if (hipMemcpy(ctx->implicit_bad, zero, sizeof zero[0], hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->stats, zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess ||
        scratch_setup(device) != MSTRUCT_OK) {
        (void)hipFree(ctx->counter);
        (void)hipFree(ctx->implicit_bad);
        (void)hipFree(ctx->stats);
        delete ctx;
        return MSTRUCT_EDEVICE;
    }
    *out = ctx;
    return MSTRUCT_OK;
}

int mstruct_destroy(mstruct_ctx* ctx) {
    if (!ctx) return MSTRUCT_EINVAL;
    DeviceGuard g(ctx->device);
    for (auto& s : ctx->slots) {
        if (s.pending) (void)hipEventSynchronize(s.done);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
    }
    if (ctx->counter) (void)hipFree(ctx->counter);
    if (ctx->implicit_bad) (void)hipFree(ctx->implicit_bad);
    if (ctx->stats) (void)hipFree(ctx->stats);
    if (ctx->wave_flags) (void)hipFree(ctx->wave_flags);
    if (ctx->wave_boxes) (void)hipFree(ctx->wave_boxes);
    mlp_free(ctx->mlp);
    delete ctx;
    return MSTRUCT_OK;
}

int mstruct_step(mstruct_ctx* ctx, const float* T_prev, const float* T_next, double dt, const mstruct_phases* ph,
                 void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    int rc = check_phases(ctx, ph);
    if (rc) return rc;
    if (!finite_pos(dt)) return fail(ctx, MSTRUCT_EINVAL, "dt must be positive and finite");
    if (ph->n > 0 && (!T_prev || !T_next)) return fail(ctx, MSTRUCT_EINVAL, "temperature array is NULL");
    DeviceGuard g(ctx->device);
    hipError_t e = launch_step(T_prev, T_next, ph->beta, ph->alpha_s, ph->alpha_m, ph->xbt, ph->n, (float)dt,
                               ctx->rd, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "step launch");
    return MSTRUCT_OK;
}

int mstruct_step_f64(mstruct_ctx* ctx, const double* T_prev, const double* T_next, double dt,
                     const mstruct_phases_f64* ph, int math, void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    if (!ph) return fail(ctx, MSTRUCT_EINVAL, "phases is NULL");
    if (ph->n < 0) return fail(ctx, MSTRUCT_EINVAL, "n < 0");
    if (ph->n > 0 && (!ph->beta || !ph->alpha_s || !ph->alpha_m || !T_prev || !T_next))
        return fail(ctx, MSTRUCT_EINVAL, "NULL array");
    if (!finite_pos(dt)) return fail(ctx, MSTRUCT_EINVAL, "dt must be positive and finite");
    if (math != MSTRUCT_F64_LIBRARY && math != MSTRUCT_F64_SYNTH && math != MSTRUCT_F64_PAPER)
        return fail(ctx, MSTRUCT_EINVAL, "bad math");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const bool cp = ctx->rd.corr_prev, ma = ctx->rd.mart_assign;
    hipError_t e =
        math == MSTRUCT_F64_LIBRARY
            ? launch_step_f64_library(T_prev, T_next, ph->beta, ph->alpha_s, ph->alpha_m, ph->n, dt, cp, ma, st)
        : math == MSTRUCT_F64_SYNTH
            ? launch_step_f64_synth(T_prev, T_next, ph->beta, ph->alpha_s, ph->alpha_m, ph->n, dt, cp, ma, st)
            : launch_step_f64_paper(T_prev, T_next, ph->beta, ph->alpha_s, ph->alpha_m, ph->n, dt, cp, ma, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "float64 step launch");
    return MSTRUCT_OK;
}

int mstruct_step_implicit(mstruct_ctx* ctx, const float* T_prev, const float* T_next, double dt, double dt_sub,
                          int max_iter, const mstruct_phases* ph, unsigned long long* unconverged, void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    int rc = check_phases(ctx, ph);
    if (rc) return rc;
    if (!finite_pos(dt)) return fail(ctx, MSTRUCT_EINVAL, "dt must be positive and finite");
    if (!finite_pos(dt_sub)) return fail(ctx, MSTRUCT_EINVAL, "dt_sub must be positive and finite");
    if (max_iter < 1 || max_iter > 1000) return fail(ctx, MSTRUCT_EINVAL, "max_iter must be in 1..1000");
    if (ph->n > 0 && (!T_prev || !T_next)) return fail(ctx, MSTRUCT_EINVAL, "temperature array is NULL");
    if (dt / dt_sub > 1e6) return fail(ctx, MSTRUCT_EINVAL, "dt / dt_sub exceeds 1e6 substeps");
    const int n_sub = substeps(dt, dt_sub);
    DeviceGuard g(ctx->device);
    hipError_t e = launch_implicit_step(T_prev, T_next, ph->beta, ph->alpha_s, ph->alpha_m, ph->xbt, ph->n,
                                        (float)(dt / n_sub), n_sub, max_iter, unconverged, ctx->rd,
                                        (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "implicit step launch");
    return MSTRUCT_OK;
}

int mstruct_temperature(mstruct_ctx* ctx, const mstruct_scan* scan, const mstruct_points* pts, double t,
                        float* T_out, void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    int rc = check_scan(ctx, scan);
    if (rc) return rc;
    if (!pts) return fail(ctx, MSTRUCT_EINVAL, "points is NULL");
    if (!isfinite(t)) return fail(ctx, MSTRUCT_EINVAL, "t must be finite");
    PointGeom pg;
    if ((rc = make_geom(ctx, pts, pts->n, pg))) return rc;
    if (pts->n > 0 && !T_out) return fail(ctx, MSTRUCT_EINVAL, "T_out is NULL");
    if (pts->n == 0) return MSTRUCT_OK;
    // the temperature call covers every point (inactive ones get T0)
    pg.first = 0;
    pg.count = pts->n;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    TableSlot* s;
    if ((rc = acquire_slot(ctx, scan->window, s))) return rc;
    build_table(s->host, scan, pts, t, 0.0, 1);
    HIP_CHECK(ctx, hipMemcpyAsync(s->dev, s->host, scan->window * sizeof(SrcRec), hipMemcpyHostToDevice, st));
    hipError_t e = launch_temperature(pg, scan->window, s->dev, ScanArgs{(float)scan->T0, (float)scan->T_clamp, ctx->rd},
                                      T_out, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "temperature launch");
    return release_slot(ctx, s, st);
}

}  // extern "C"

namespace {

// Sizes of one fused call: its table (records of n_steps + 1 time points x
// W slots, then (first, count) int32 pairs of each launch's envelopes, then
// at most (K + 1) W envelope records per launch) and its waves of 64 points.
struct FusedPlan {
    int W;
    int64_t n_launches, n_waves;
    size_t recs, fc_recs, env_cap;
    size_t table() const { return recs + fc_recs + env_cap; }
};

// steps per launch: K, or in SURROGATE mode (K = the network's block) the
// most whole blocks that fit in 64 steps
int launch_steps(int K, int mode) { return mode == MSTRUCT_MODE_SURROGATE ? K * (64 / K) : K; }

FusedPlan fused_plan(const mstruct_scan* scan, const PointGeom& pg, int64_t n_steps, int K) {
    FusedPlan p;
    p.W = scan->window;
    p.n_launches = (n_steps + K - 1) / K;
    p.n_waves = (pg.count + kWave - 1) / kWave;
    p.recs = (size_t)(n_steps + 1) * p.W;
    p.fc_recs = ((size_t)p.n_launches * 2 * sizeof(int32_t) + sizeof(SrcRec) - 1) / sizeof(SrcRec);
    p.env_cap = (size_t)p.n_launches * (K + 1) * p.W;
    return p;
}

// The buffers a fused call works in: the table's host staging and its
// device copy (cap records each), and the wave flags (n_waves bytes of rest
// flags, then still flags for chunks of `chunk` launches; flags == nullptr:
// none) with the waves' boxes on an index list.
//
// With wave flags, calls also list the waves each slot launch steps (4 bytes
// per wave, and two counts: list_bytes in all).
struct FusedBufs {
    SrcRec* host = nullptr;
    SrcRec* dev = nullptr;
    size_t cap = 0;
    uint8_t* flags = nullptr;
    int64_t chunk = 0;
    GridBox* boxes = nullptr;
    uint32_t* cand = nullptr;
    unsigned* cand_counts = nullptr;
};

size_t round256(size_t n) { return (n + 255) & ~(size_t)255; }

// bytes of a launch's wave list and its two counts (a call has fewer than
// 2^31 points, so its waves are numbered in 32 bits)
size_t list_bytes(int64_t n_waves) { return round256((size_t)n_waves * sizeof(uint32_t)) + 256; }

void place_list(FusedBufs& b, uint8_t* at, int64_t n_waves) {
    b.cand = reinterpret_cast<uint32_t*>(at);
    b.cand_counts = reinterpret_cast<unsigned*>(at + round256((size_t)n_waves * sizeof(uint32_t)));
}

// Argument checks shared by the fused entry points; fills pg.  Returns
// MSTRUCT_OK, an error status, or 1 when there is nothing to do.
int fused_check(mstruct_ctx* ctx, const mstruct_scan* scan, const mstruct_points* pts, double t0, double dt,
                int64_t n_steps, int K, int mode, const mstruct_phases* ph, PointGeom& pg) {
    if (!ctx) return MSTRUCT_EINVAL;
    int rc = check_phases(ctx, ph);
    if (rc) return rc;
    if ((rc = check_scan(ctx, scan))) return rc;
    if (!finite_pos(dt) || !isfinite(t0)) return fail(ctx, MSTRUCT_EINVAL, "bad t0 or dt");
    if (n_steps < 0) return fail(ctx, MSTRUCT_EINVAL, "n_steps < 0");
    if (K < 1 || K > 64) return fail(ctx, MSTRUCT_EINVAL, "K must be in 1..64");
    if (mode != MSTRUCT_MODE_PLAIN && mode != MSTRUCT_MODE_SURROGATE && mode != MSTRUCT_MODE_IMPLICIT)
        return fail(ctx, MSTRUCT_EINVAL, "bad mode");
    if (mode == MSTRUCT_MODE_IMPLICIT && dt / kImplicitDtSub > 1e6)
        return fail(ctx, MSTRUCT_EINVAL, "dt / 0.01 s exceeds 1e6 substeps");
    if ((rc = make_geom(ctx, pts, ph->n, pg))) return rc;
    choose_wave_shape(ctx, scan, pts, t0, t0 + (double)n_steps * dt, pg);
    if (mode == MSTRUCT_MODE_SURROGATE && ph->xbt)
        return fail(ctx, MSTRUCT_EUNSUPPORTED, "surrogate mode does not carry the tracked X~beta (xbt)");
    if (mode == MSTRUCT_MODE_SURROGATE && !ctx->mlp.ready)
        return fail(ctx, MSTRUCT_ESTATE, "surrogate mode needs network parameters (mstruct_mlp_set_params)");
    if (mode == MSTRUCT_MODE_SURROGATE && (ctx->rd.corr_prev || ctx->rd.mart_assign))
        return fail(ctx, MSTRUCT_EUNSUPPORTED, "surrogate mode runs with the default readings only");
    if (n_steps == 0 || pg.count == 0) return 1;
    return MSTRUCT_OK;
}

// The body of a fused call: scan table and launch envelopes built on the
// host into b.host, uploaded to b.dev (then `uploaded`, if given, is
// recorded on the stream), the still-flag pre-passes and the launches of K
// steps (in SURROGATE mode in network blocks of Ks steps).  Nothing is
// enqueued if the table does not fit.
int fused_run(mstruct_ctx* ctx, const mstruct_scan* scan, const mstruct_points* pts, const PointGeom& pg,
              const FusedPlan& p, double t0, double dt, int64_t n_steps, int K, int Ks, int mode,
              const mstruct_phases* ph, const FusedBufs& b, hipEvent_t uploaded, hipStream_t st) {
    const int W = p.W;
    if (p.recs + p.fc_recs > b.cap) return fail(ctx, MSTRUCT_EINVAL, "scan table larger than the table buffer");
    build_table(b.host, scan, pts, t0, dt, n_steps + 1);
    int32_t* fc_host = reinterpret_cast<int32_t*>(b.host + p.recs);
    const int32_t* fc_dev = reinterpret_cast<const int32_t*>(b.dev + p.recs);
    EnvRec* env_host = reinterpret_cast<EnvRec*>(b.host + p.recs + p.fc_recs);
    const EnvRec* env_dev = reinterpret_cast<const EnvRec*>(b.dev + p.recs + p.fc_recs);
    const int64_t n_env = build_envelopes(env_host, (int64_t)(b.cap - p.recs - p.fc_recs), fc_host, b.host, scan, t0,
                                          dt, n_steps, K);
    if (n_env < 0) return fail(ctx, MSTRUCT_EINVAL, "launch envelopes larger than the table buffer");
    HIP_CHECK(ctx, hipMemcpyAsync(b.dev, b.host, (p.recs + p.fc_recs + (size_t)n_env) * sizeof(SrcRec),
                                  hipMemcpyHostToDevice, st));
    if (uploaded) HIP_CHECK(ctx, hipEventRecord(uploaded, st));
    const ScanArgs sa{(float)scan->T0, (float)scan->T_clamp, ctx->rd};
    const bool wave_flags = b.flags != nullptr;
    const int64_t n_waves = p.n_waves, n_launches = p.n_launches, chunk = b.chunk;
    if (mode == MSTRUCT_MODE_SURROGATE) {
        hipError_t e = surrogate_prepare(ctx->mlp, n_waves, st);
        if (e != hipSuccess) return hip_fail(ctx, e, "surrogate records");
    }
    if (mode != MSTRUCT_MODE_IMPLICIT && wave_flags && b.cand) {
        // each chunk of launches in one persistent kernel (fused_plain_call_kernel; SURROGATE:
        // fused_surrogate_call_kernel and surrogate_resume_call_kernel); IMPLICIT calls, whose cool-downs
        // step most waves in every launch, keep one kernel per launch: in one kernel per chunk the last
        // waves run whole chunks alone (cool-down workload 194 -> 216 ms)
        for (int64_t l0 = 0; l0 < n_launches; l0 += chunk) {
            const int64_t nl = (n_launches - l0) < chunk ? (n_launches - l0) : chunk;
            const GridBox* boxes = pts->index ? b.boxes : nullptr;
            hipError_t e = hipSuccess;
            if (l0 == 0 && boxes) e = launch_wave_boxes(pg, n_waves, b.boxes, st);
            if (e == hipSuccess)
                e = launch_still_flags(pg, env_dev, fc_dev, l0, nl, n_waves, fminf(sa.T0, sa.Tclamp), boxes,
                                       b.flags + n_waves, st);
            float* beta = l0 + nl == n_launches ? ph->beta : nullptr;
            unsigned long long* stats = ctx->count_waves ? ctx->stats : nullptr;
            if (e == hipSuccess && mode == MSTRUCT_MODE_PLAIN)
                e = launch_fused_plain_call(pg, W, b.dev, env_dev, fc_dev, b.flags + n_waves, b.flags, n_waves, l0,
                                            nl, K, n_steps, (float)dt, sa, beta, ph->alpha_s, ph->alpha_m, b.cand,
                                            b.cand_counts, stats, st);
            else if (e == hipSuccess)
                e = launch_surrogate_call(ctx->mlp, pg, W, b.dev, env_dev, fc_dev, b.flags + n_waves, b.flags, n_waves,
                                          l0, nl, K, Ks, n_steps, (float)dt, sa, beta, ph->alpha_s, ph->alpha_m, b.cand,
                                          b.cand_counts, stats, st);
            if (e != hipSuccess) return hip_fail(ctx, e, "fused call launch");
        }
        return MSTRUCT_OK;
    }
    const bool list = wave_flags && b.cand;
    if (list) {
        hipError_t e = launch_clear_counts(b.cand_counts, st);
        if (e != hipSuccess) return hip_fail(ctx, e, "wave list counts");
    }
    for (int64_t s0 = 0; s0 < n_steps; s0 += K) {
        const int Kb = (int)((n_steps - s0) < K ? (n_steps - s0) : K);
        const bool last = s0 + Kb >= n_steps;
        // beta is written by the last launch only (no kernel reads it)
        float* beta = last ? ph->beta : nullptr;
        hipError_t e;
        const int64_t li = s0 / K;
        uint8_t* below = nullptr;
        if (wave_flags) {
            below = b.flags + n_waves * (1 + li % chunk);
            if (li % chunk == 0) {
                const int64_t nl = (n_launches - li) < chunk ? (n_launches - li) : chunk;
                const GridBox* boxes = pts->index ? b.boxes : nullptr;
                hipError_t fe = hipSuccess;
                if (li == 0 && boxes) fe = launch_wave_boxes(pg, n_waves, b.boxes, st);
                if (fe == hipSuccess)
                    fe = launch_still_flags(pg, env_dev, fc_dev, li, nl, n_waves, fminf(sa.T0, sa.Tclamp), boxes,
                                            b.flags + n_waves, st);
                if (fe != hipSuccess) return hip_fail(ctx, fe, "still flags launch");
            }
        }
        const bool use_list = list;
        const EnvSet es{env_dev + fc_host[2 * li], ctx->skip_cold ? fc_host[2 * li + 1] : -1, below,
                        wave_flags ? b.flags : nullptr, n_waves, li > 0, ctx->count_waves ? ctx->stats : nullptr,
                        use_list ? b.cand : nullptr, use_list ? b.cand_counts + (li & 1) : nullptr,
                        use_list ? b.cand_counts + ((li + 1) & 1) : nullptr};
        if (use_list) {
            hipError_t le = li == 0 ? launch_first_candidates(pg, es, fminf(sa.T0, sa.Tclamp), beta, ph->alpha_s,
                                                              ph->alpha_m, st)
                                    : launch_candidates(pg, es, fminf(sa.T0, sa.Tclamp), beta, st);
            if (le != hipSuccess) return hip_fail(ctx, le, "wave list launch");
        }
        if (mode == MSTRUCT_MODE_PLAIN) {
            e = launch_fused_plain(pg, W, b.dev + s0 * W, es, Kb, (float)dt, sa, beta, ph->alpha_s, ph->alpha_m,
                                   ph->xbt, st);
        } else if (mode == MSTRUCT_MODE_IMPLICIT) {
            const int n_sub = substeps(dt, kImplicitDtSub);
            e = launch_fused_implicit(pg, W, b.dev + s0 * W, es, Kb, (float)(dt / n_sub), n_sub, kImplicitMaxIter,
                                      sa, beta, ph->alpha_s, ph->alpha_m, ph->xbt, ctx->implicit_bad, st);
        } else
            e = launch_surrogate(ctx->mlp, pg, W, b.dev + s0 * W, es, Kb, Ks, (float)dt, sa, beta, ph->alpha_s,
                                 ph->alpha_m, li, st);
        if (e != hipSuccess) return hip_fail(ctx, e, "fused launch");
    }
    return MSTRUCT_OK;
}

// ---- the device array of the allocation-free fused call ----
// One array per GPU, for the life of the process (a static __device__
// variable; the host code reaches it only through the address
// hipGetSymbolAddress gives on each device): the scan table (kScratchTable
// bytes), then the waves' boxes and the wave flags.  Its table is uploaded
// from a static host array of the same size, one call at a time.
constexpr size_t kScratchTable = (size_t)4 << 20;
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

struct ScratchState {
    std::mutex lock;                             // the host staging array, one call at a time
    uint8_t* dev[kScratchDevices] = {};          // address of `scratch` on each device (nullptr: not set up)
    hipEvent_t uploaded[kScratchDevices] = {};   // the last upload from the staging array on each device
    hipEvent_t pending = nullptr;                // the last upload that may still read the staging array
};
ScratchState g_scratch;
alignas(256) SrcRec g_scratch_stage[kScratchTable / sizeof(SrcRec)];

// once per device, with the device current (called by mstruct_init)
int scratch_setup(int device) {
    if (device >= kScratchDevices) return MSTRUCT_OK;  // the allocation-free call is not available there
    std::lock_guard<std::mutex> g(g_scratch.lock);
    if (g_scratch.dev[device]) return MSTRUCT_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MSTRUCT_EDEVICE;
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return MSTRUCT_EDEVICE;
    g_scratch.uploaded[device] = ev;
    g_scratch.dev[device] = static_cast<uint8_t*>(ptr);
    return MSTRUCT_OK;
}

}  // namespace

extern "C" {

int mstruct_fused_scan_steps(mstruct_ctx* ctx, const mstruct_scan* scan, const mstruct_points* pts, double t0,
                             double dt, int64_t n_steps, int K, int mode, const mstruct_phases* ph, void* stream) {
    PointGeom pg;
    int rc = fused_check(ctx, scan, pts, t0, dt, n_steps, K, mode, ph, pg);
    if (rc) return rc > 0 ? MSTRUCT_OK : rc;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const int Kl = launch_steps(K, mode);
    const FusedPlan p = fused_plan(scan, pg, n_steps, Kl);
    FusedBufs b;
    // Wave flags (one point per lane, 64 per wave): rest flags kept by the
    // fused kernels, then still flags for chunks of launches from a box
    // pre-pass (on an index list the boxes of the waves are computed first).
    // Not with the tracked X~beta, whose store every launch takes.
    if (ctx->skip_cold && !ph->xbt) {
        int64_t chunk = kWaveFlagBudget / p.n_waves;
        chunk = chunk < 1 ? 1 : (chunk > p.n_launches ? p.n_launches : chunk);
        const size_t flag_bytes = round256((size_t)p.n_waves * (size_t)(1 + chunk));
        const size_t need = flag_bytes + list_bytes(p.n_waves);
        if (ctx->wave_flags_cap < need) {
            HIP_CHECK(ctx, hipStreamSynchronize(st));
            if (ctx->wave_flags) HIP_CHECK(ctx, hipFree(ctx->wave_flags));
            ctx->wave_flags = nullptr;
            ctx->wave_flags_cap = 0;
            if (hipMalloc((void**)&ctx->wave_flags, need) != hipSuccess) {
                ctx->wave_flags = nullptr;
                return fail(ctx, MSTRUCT_ENOMEM, "wave flag allocation failed");
            }
            ctx->wave_flags_cap = need;
        }
        const size_t n_boxes = (size_t)(p.n_waves + wave_groups(p.n_waves));
        if (pts->index && ctx->wave_boxes_cap < n_boxes) {
            HIP_CHECK(ctx, hipStreamSynchronize(st));
            if (ctx->wave_boxes) HIP_CHECK(ctx, hipFree(ctx->wave_boxes));
            ctx->wave_boxes = nullptr;
            ctx->wave_boxes_cap = 0;
            if (hipMalloc((void**)&ctx->wave_boxes, n_boxes * sizeof(GridBox)) != hipSuccess) {
                ctx->wave_boxes = nullptr;
                return fail(ctx, MSTRUCT_ENOMEM, "wave box allocation failed");
            }
            ctx->wave_boxes_cap = n_boxes;
        }
        b.flags = ctx->wave_flags;
        b.chunk = chunk;
        b.boxes = ctx->wave_boxes;
        place_list(b, ctx->wave_flags + flag_bytes, p.n_waves);
    }
    TableSlot* s;
    if ((rc = acquire_slot(ctx, p.table(), s))) return rc;
    b.host = s->host;
    b.dev = s->dev;
    b.cap = s->cap;
    rc = fused_run(ctx, scan, pts, pg, p, t0, dt, n_steps, Kl, K, mode, ph, b, nullptr, st);
    const int rc2 = release_slot(ctx, s, st);
    return rc ? rc : rc2;
}

int mstruct_fused_scan_steps_noalloc(mstruct_ctx* ctx, const mstruct_scan* scan, const mstruct_points* pts,
                                     double t0, double dt, int64_t n_steps, int K, int mode, const mstruct_phases* ph,
                                     void* stream) {
    if (ctx && mode == MSTRUCT_MODE_SURROGATE)
        return fail(ctx, MSTRUCT_EUNSUPPORTED, "the allocation-free call runs PLAIN and IMPLICIT modes only");
    PointGeom pg;
    int rc = fused_check(ctx, scan, pts, t0, dt, n_steps, K, mode, ph, pg);
    if (rc < 0) return rc;
    const FusedPlan p = rc > 0 ? FusedPlan{} : fused_plan(scan, pg, n_steps, K);
    // the table must fit; the exact envelope count is checked as it is built
    if (rc == 0 && (p.recs + p.fc_recs) * sizeof(SrcRec) > kScratchTable) {
        char buf[160];
        snprintf(buf, sizeof buf, "%zu table records exceed the allocation-free limit of %zu",
                 p.recs + p.fc_recs, kScratchTable / sizeof(SrcRec));
        return fail(ctx, MSTRUCT_EINVAL, "%s", buf);
    }
    if (ctx->device >= kScratchDevices || !g_scratch.dev[ctx->device])
        return fail(ctx, MSTRUCT_EUNSUPPORTED, "no allocation-free array on this device");
    if (rc > 0) return MSTRUCT_OK;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    uint8_t* base = g_scratch.dev[ctx->device];
    FusedBufs b;
    b.host = g_scratch_stage;
    b.dev = reinterpret_cast<SrcRec*>(base);
    b.cap = kScratchTable / sizeof(SrcRec);
    // wave boxes (index lists) and flags in the rest of the array, as many
    // launches of still flags per chunk as fit; without room for one launch
    // the call runs without wave flags (the same results bit for bit)
    if (ctx->skip_cold && !ph->xbt) {
        const size_t box_bytes =
            pts->index ? round256((size_t)(p.n_waves + wave_groups(p.n_waves)) * sizeof(GridBox)) : 0;
        const size_t lb = list_bytes(p.n_waves);
        const size_t room = kScratchBytes - kScratchTable;
        const size_t used = box_bytes + lb + 256;
        const int64_t per_wave = used < room ? (int64_t)((room - used) / (size_t)p.n_waves) : 0;
        int64_t chunk = per_wave - 1;
        if (chunk >= 1) {
            b.boxes = pts->index ? reinterpret_cast<GridBox*>(base + kScratchTable) : nullptr;
            place_list(b, base + kScratchTable + box_bytes, p.n_waves);
            b.flags = base + kScratchTable + box_bytes + lb;
            b.chunk = chunk > p.n_launches ? p.n_launches : chunk;
        }
    }
    std::lock_guard<std::mutex> lk(g_scratch.lock);
    // the staging array is rewritten only after the last upload from it is done
    if (g_scratch.pending) HIP_CHECK(ctx, hipEventSynchronize(g_scratch.pending));
    g_scratch.pending = nullptr;
    rc = fused_run(ctx, scan, pts, pg, p, t0, dt, n_steps, K, K, mode, ph, b, g_scratch.uploaded[ctx->device], st);
    // (if the upload was not enqueued, the event holds an earlier, harmless record)
    g_scratch.pending = g_scratch.uploaded[ctx->device];
    return rc;
}

int mstruct_set_option(mstruct_ctx* ctx, int option, int value) {
    if (!ctx) return MSTRUCT_EINVAL;
    switch (option) {
        case MSTRUCT_OPTION_SKIP_COLD_WAVES: ctx->skip_cold = value != 0; return MSTRUCT_OK;
        case MSTRUCT_OPTION_COUNT_WAVES: ctx->count_waves = value != 0; return MSTRUCT_OK;
        case MSTRUCT_OPTION_TILE_WAVES: ctx->tile_waves = value != 0; return MSTRUCT_OK;
        case MSTRUCT_OPTION_WAVE_TILE_WIDTH:
            if (value != 0 && (value < 1 || value > 64 || (value & (value - 1))))
                return fail(ctx, MSTRUCT_EINVAL, "tile width must be 0 or a power of two in 1..64");
            ctx->tile_width = value;
            return MSTRUCT_OK;
        default: return fail(ctx, MSTRUCT_EINVAL, "unknown option");
    }
}

int mstruct_implicit_unconverged(mstruct_ctx* ctx, int64_t* count, int reset, void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    if (!count) return fail(ctx, MSTRUCT_EINVAL, "count is NULL");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    unsigned long long h = 0;
    HIP_CHECK(ctx, hipMemcpyAsync(&h, ctx->implicit_bad, sizeof h, hipMemcpyDeviceToHost, st));
    if (reset) {
        const unsigned long long zero = 0;
        HIP_CHECK(ctx, hipMemcpyAsync(ctx->implicit_bad, &zero, sizeof zero, hipMemcpyHostToDevice, st));
    }
    HIP_CHECK(ctx, hipStreamSynchronize(st));
    *count = (int64_t)h;
    return MSTRUCT_OK;
}

int mstruct_wave_counts(mstruct_ctx* ctx, int64_t* counts, int reset, void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    if (!counts) return fail(ctx, MSTRUCT_EINVAL, "counts is NULL");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    unsigned long long h[kStatCount] = {};
    HIP_CHECK(ctx, hipMemcpyAsync(h, ctx->stats, sizeof h, hipMemcpyDeviceToHost, st));
    if (reset) {
        const unsigned long long zero[kStatCount] = {};
        HIP_CHECK(ctx, hipMemcpyAsync(ctx->stats, zero, sizeof zero, hipMemcpyHostToDevice, st));
    }
    HIP_CHECK(ctx, hipStreamSynchronize(st));
    for (int i = 0; i < kStatCount; ++i) counts[i] = (int64_t)h[i];
    return MSTRUCT_OK;
}

int mstruct_gather(mstruct_ctx* ctx, const float* src, const int64_t* idx, int64_t m, float* dst, void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    if (m < 0) return fail(ctx, MSTRUCT_EINVAL, "m < 0");
    if (m > 0 && (!src || !idx || !dst)) return fail(ctx, MSTRUCT_EINVAL, "NULL array");
    DeviceGuard g(ctx->device);
    hipError_t e = launch_gather(src, idx, m, dst, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "gather launch");
    return MSTRUCT_OK;
}

int mstruct_check_invariants(mstruct_ctx* ctx, const mstruct_phases* ph, const float* T, float tol,
                             int64_t* violations, void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    int rc = check_phases(ctx, ph);
    if (rc) return rc;
    if (!violations) return fail(ctx, MSTRUCT_EINVAL, "violations is NULL");
    if (!(tol >= 0.0f)) return fail(ctx, MSTRUCT_EINVAL, "tol must be >= 0");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const unsigned long long zero = 0;
    HIP_CHECK(ctx, hipMemcpyAsync(ctx->counter, &zero, sizeof zero, hipMemcpyHostToDevice, st));
    hipError_t e = launch_invariants(ph->beta, ph->alpha_s, ph->alpha_m, T, ph->n, tol, ctx->counter, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "invariants launch");
    unsigned long long h = 0;
    HIP_CHECK(ctx, hipMemcpyAsync(&h, ctx->counter, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_CHECK(ctx, hipStreamSynchronize(st));
    *violations = (int64_t)h;
    return MSTRUCT_OK;
}

}  // extern "C"

// ---- learned surrogate and correction entry points ----
extern "C" {

int mstruct_correct(mstruct_ctx* ctx, const float* T, const mstruct_phases* ph, void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    int rc = check_phases(ctx, ph);
    if (rc) return rc;
    if (ph->n > 0 && !T) return fail(ctx, MSTRUCT_EINVAL, "T is NULL");
    DeviceGuard g(ctx->device);
    hipError_t e = launch_correct(T, ph->beta, ph->alpha_s, ph->alpha_m, ph->n, ctx->rd.mart_assign,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "correct launch");
    return MSTRUCT_OK;
}

int mstruct_mlp_set_params(mstruct_ctx* ctx, const float* params, const float* in_mean, const float* in_scale,
                           const float* out_scale, const float* indicator) {
    if (!ctx) return MSTRUCT_EINVAL;
    if (!params || !in_mean || !in_scale || !out_scale) return fail(ctx, MSTRUCT_EINVAL, "NULL argument");
    for (int i = 0; i < kMlpParams; ++i)
        if (!isfinite(params[i])) return fail(ctx, MSTRUCT_EINVAL, "non-finite parameter");
    MlpNorm nrm{};
    for (int k = 0; k < kMlpIn; ++k) {
        if (!isfinite(in_mean[k]) || !(in_scale[k] > 0.0f) || !isfinite(in_scale[k]))
            return fail(ctx, MSTRUCT_EINVAL, "bad input normalisation");
        nrm.in_mean[k] = in_mean[k];
        nrm.in_inv_scale[k] = 1.0f / in_scale[k];
    }
    for (int k = 0; k < kMlpOut; ++k) {
        if (!(out_scale[k] > 0.0f) || !isfinite(out_scale[k])) return fail(ctx, MSTRUCT_EINVAL, "bad output scale");
        nrm.out_scale[k] = out_scale[k];
    }
    // error indicator: default bands around the martensite start (848 K),
    // the beta transus / regularisation range (935..1373 K) and melting
    const float def[4] = {823.0f, 1398.0f, 1853.0f, 50.0f};
    const float* ind = indicator ? indicator : def;
    for (int k = 0; k < 4; ++k)
        if (!isfinite(ind[k])) return fail(ctx, MSTRUCT_EINVAL, "non-finite indicator threshold");
    if (!(ind[3] >= 0.0f)) return fail(ctx, MSTRUCT_EINVAL, "dT_max must be >= 0");
    nrm.T_cold = ind[0];
    nrm.T_hot_lo = ind[1];
    nrm.T_hot_hi = ind[2];
    nrm.dT_max = ind[3];
    DeviceGuard g(ctx->device);
    MlpState& s = ctx->mlp;
    HIP_CHECK(ctx, mlp_alloc(s));
    HIP_CHECK(ctx, hipDeviceSynchronize());
    HIP_CHECK(ctx, hipMemcpy(s.master, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice));
    HIP_CHECK(ctx, hipMemset(s.adam_m, 0, kMlpParams * sizeof(float)));
    HIP_CHECK(ctx, hipMemset(s.adam_v, 0, kMlpParams * sizeof(float)));
    s.adam_t = 0;
    s.norm = nrm;
    HIP_CHECK(ctx, mlp_pack(s, nullptr));
    HIP_CHECK(ctx, hipDeviceSynchronize());
    s.ready = true;
    return MSTRUCT_OK;
}

int mstruct_mlp_get_params(mstruct_ctx* ctx, float* params) {
    if (!ctx) return MSTRUCT_EINVAL;
    if (!params) return fail(ctx, MSTRUCT_EINVAL, "NULL argument");
    if (!ctx->mlp.ready) return fail(ctx, MSTRUCT_ESTATE, "no network parameters set");
    DeviceGuard g(ctx->device);
    HIP_CHECK(ctx, hipDeviceSynchronize());
    HIP_CHECK(ctx, hipMemcpy(params, ctx->mlp.master, kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
    return MSTRUCT_OK;
}

int mstruct_mlp_forward(mstruct_ctx* ctx, const float* X, int64_t B, float* Y, void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    if (B < 0) return fail(ctx, MSTRUCT_EINVAL, "B < 0");
    if (B > 0 && (!X || !Y)) return fail(ctx, MSTRUCT_EINVAL, "NULL array");
    if (!ctx->mlp.ready) return fail(ctx, MSTRUCT_ESTATE, "no network parameters set");
    DeviceGuard g(ctx->device);
    hipError_t e = mlp_forward(ctx->mlp, X, B, Y, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "mlp forward launch");
    return MSTRUCT_OK;
}

int mstruct_mlp_grad(mstruct_ctx* ctx, const float* X, const float* Y, int64_t B, float* grad, float* loss,
                     void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    if (B < 1) return fail(ctx, MSTRUCT_EINVAL, "B must be >= 1");
    if (!X || !Y || !grad || !loss) return fail(ctx, MSTRUCT_EINVAL, "NULL array");
    if (!ctx->mlp.ready) return fail(ctx, MSTRUCT_ESTATE, "no network parameters set");
    DeviceGuard g(ctx->device);
    hipError_t e = mlp_grad(ctx->mlp, X, Y, B, grad, loss, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "mlp gradient launch");
    return MSTRUCT_OK;
}

int mstruct_mlp_train_step(mstruct_ctx* ctx, const float* X, const float* Y, int64_t B, float lr, float* loss,
                           void* stream) {
    if (!ctx) return MSTRUCT_EINVAL;
    if (B < 1) return fail(ctx, MSTRUCT_EINVAL, "B must be >= 1");
    if (!X || !Y) return fail(ctx, MSTRUCT_EINVAL, "NULL array");
    if (!(lr > 0.0f) || !isfinite(lr)) return fail(ctx, MSTRUCT_EINVAL, "lr must be positive");
    if (!ctx->mlp.ready) return fail(ctx, MSTRUCT_ESTATE, "no network parameters set");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    MlpState& s = ctx->mlp;
    hipError_t e = mlp_grad(s, X, Y, B, s.grad, s.loss, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "mlp gradient launch");
    if ((e = mlp_adam(s, lr, st)) != hipSuccess) return hip_fail(ctx, e, "adam launch");
    if (loss) HIP_CHECK(ctx, hipMemcpyAsync(loss, s.loss, sizeof(float), hipMemcpyDeviceToDevice, st));
    return MSTRUCT_OK;
}

}  // extern "C"
