// Phase-update kernels for gfx950: the plain explicit step over temperature
// arrays (HBM-bound streaming), the temperature field of a scan, and the fused
// kernel that keeps each point's state in registers for K steps while
// evaluating the temperature analytically (VALU-bound).
#include "fused.h"

namespace mstruct {

constexpr int kBlock = 256;
// points per lane of the fused grid kernel, a build-time choice: 1 (the
// wave flags, slot kernels and still shortcuts assume it); 2 or 4 advance
// independent points together for instruction-level parallelism, without
// those shortcuts
#ifndef FUSED_PPT
#define FUSED_PPT 1
#endif
typedef float vf4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// plain step: Algorithm 1's loop over points with the local explicit step of
// Algorithm 2; reads alpha_s, alpha_m, T^n, T^{n+1} and writes the three
// fractions (28 bytes per point).  VEC: four consecutive points per thread
// with 16-byte accesses (all five arrays 16-byte aligned).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void step_point(float Tp, float Tn, float& b, float& a, float& m, float dt, Readings rd) {
    float alo = 0.0f, mlo = 0.0f;
    b = explicit_step<false>(a, m, alo, mlo, Tp, alpha_eq(Tp), Tn, alpha_eq(Tn), dt, rd);
}

template <bool VEC>
__global__ __launch_bounds__(kBlock) void step_kernel(const float* __restrict__ Tp, const float* __restrict__ Tn,
                                                     float* __restrict__ beta, float* __restrict__ as,
                                                     float* __restrict__ am, int64_t n, float dt, Readings rd) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (VEC) {
        const int64_t i = 4 * g;
        if (i + 3 < n) {
            const vf4 tp = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(Tp) + g);
            const vf4 tn = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(Tn) + g);
            vf4 a = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(as) + g);
            vf4 m = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(am) + g);
            vf4 b;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                float ac = a[c], mc = m[c], bc;
                step_point(tp[c], tn[c], bc, ac, mc, dt, rd);
                a[c] = ac;
                m[c] = mc;
                b[c] = bc;
            }
            __builtin_nontemporal_store(a, reinterpret_cast<vf4*>(as) + g);
            __builtin_nontemporal_store(m, reinterpret_cast<vf4*>(am) + g);
            __builtin_nontemporal_store(b, reinterpret_cast<vf4*>(beta) + g);
        } else {
            for (int64_t j = i; j < n; ++j) {
                float a = as[j], m = am[j], b;
                step_point(Tp[j], Tn[j], b, a, m, dt, rd);
                as[j] = a;
                am[j] = m;
                beta[j] = b;
            }
        }
    } else {
        if (g < n) {
            float a = as[g], m = am[g], b;
            step_point(Tp[g], Tn[g], b, a, m, dt, rd);
            as[g] = a;
            am[g] = m;
            beta[g] = b;
        }
    }
}

// the explicit step with the tracked X~beta side value (float64 per point)
__global__ __launch_bounds__(kBlock) void step_tracked_kernel(const float* __restrict__ Tp,
                                                             const float* __restrict__ Tn, float* __restrict__ beta,
                                                             float* __restrict__ as, float* __restrict__ am,
                                                             double* __restrict__ xbv, int64_t n, float dt,
                                                             Readings rd) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= n) return;
    float a = as[g], m = am[g], alo = 0.0f, mlo = 0.0f;
    double xb = track_check(xbv[g], a, m);
    const float tp = Tp[g], tn = Tn[g];
    beta[g] = explicit_step_tracked<false>(a, m, alo, mlo, xb, tp, alpha_eq(tp), tn, alpha_eq(tn), dt, rd);
    as[g] = a;
    am[g] = m;
    xbv[g] = xb;
}

hipError_t launch_step(const float* Tp, const float* Tn, float* beta, float* as, float* am, double* xb, int64_t n,
                       float dt, Readings rd, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (xb) {
        hipLaunchKernelGGL(step_tracked_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, Tp,
                           Tn, beta, as, am, xb, n, dt, rd);
        return hipGetLastError();
    }
    const uintptr_t align = (uintptr_t)Tp | (uintptr_t)Tn | (uintptr_t)beta | (uintptr_t)as | (uintptr_t)am;
    if ((align & 15) == 0) {
        const int64_t threads = (n + 3) / 4;
        const int64_t blocks = (threads + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(step_kernel<true>, dim3((unsigned)blocks), dim3(kBlock), 0, st, Tp, Tn, beta, as, am,
                           n, dt, rd);
    } else {
        const int64_t blocks = (n + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(step_kernel<false>, dim3((unsigned)blocks), dim3(kBlock), 0, st, Tp, Tn, beta, as, am,
                           n, dt, rd);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// implicit step: n_sub equal substeps of length h with T linear in time, the
// Crank-Nicolson fixed-point step on each (28 bytes per point like the
// explicit step; the iteration makes it compute-heavier).  Substeps whose
// iteration hit max_iter are counted, one atomic per wave.
// ---------------------------------------------------------------------------
// TRACK: with the tracked X~beta side value (float64 per point)
template <bool TRACK>
__global__ __launch_bounds__(kBlock) void implicit_step_kernel(const float* __restrict__ Tp,
                                                              const float* __restrict__ Tn,
                                                              float* __restrict__ beta, float* __restrict__ as,
                                                              float* __restrict__ am, double* __restrict__ xbv,
                                                              int64_t n, float h, int n_sub, int max_iter,
                                                              unsigned long long* __restrict__ unconverged,
                                                              bool assign) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int bad = 0;
    if (g < n) {
        float a = as[g], m = am[g], b = 0.0f, alo = 0.0f, mlo = 0.0f;
        double xb = TRACK ? track_check(xbv[g], a, m) : 0.0;
        const float T0 = Tp[g], dT = Tn[g] - T0;
        const float inv = 1.0f / (float)n_sub;
        float Ta = T0;
        for (int s = 0; s < n_sub; ++s) {
            const float Tb = (s + 1 == n_sub) ? Tn[g] : fmaf(dT, (float)(s + 1) * inv, T0);
            const int it = TRACK ? implicit_step_tracked<false>(a, m, alo, mlo, xb, b, Ta, Tb, h, max_iter, assign)
                                 : implicit_step<false>(a, m, alo, mlo, b, Ta, Tb, h, max_iter, assign);
            if (it < 0) ++bad;
            Ta = Tb;
        }
        as[g] = a;
        am[g] = m;
        beta[g] = b;
        if (TRACK) xbv[g] = xb;
    }
    if (unconverged) {
        // sum of the per-lane counts over the wave (counts are small)
        int total = bad;
        for (int o = 32; o > 0; o >>= 1) total += __shfl_xor(total, o);
        if ((threadIdx.x & 63) == 0 && total) atomicAdd(unconverged, (unsigned long long)total);
    }
}

hipError_t launch_implicit_step(const float* Tp, const float* Tn, float* beta, float* as, float* am, double* xb,
                                int64_t n, float h, int n_sub, int max_iter, unsigned long long* unconverged,
                                Readings rd, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    if (xb)
        hipLaunchKernelGGL(implicit_step_kernel<true>, grid, block, 0, st, Tp, Tn, beta, as, am, xb, n, h, n_sub,
                           max_iter, unconverged, rd.mart_assign);
    else
        hipLaunchKernelGGL(implicit_step_kernel<false>, grid, block, 0, st, Tp, Tn, beta, as, am, xb, n, h, n_sub,
                           max_iter, unconverged, rd.mart_assign);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// temperature field at one time point
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kBlock) void temperature_kernel(PointGeom pg, const SrcRec* __restrict__ rec,
                                                            ScanArgs sa, float* __restrict__ T) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= pg.count) return;
    const int64_t local = pg.first + g;
    int gi, gj, gk;
    decode_point(pg, local, gi, gj, gk);
    T[local] = (gk < pg.k0) ? sa.T0 : scan_temperature<W>(rec, gi, gj, gk, sa.T0, sa.Tclamp, pg.r2min, pg.roff);
}

// the box of grid positions holding the points g0 .. g1 of pg's wave order
// (a box grid): part of one row, or whole rows of one plane, or whole
// planes; on a tiled grid (g0 and g1 + 1 multiples of 64) part of one row of
// tiles, from the first tile's first point to the last tile's last, or whole
// rows of tiles of one plane, or whole planes
__device__ __forceinline__ GridBox range_box(const PointGeom& pg, int64_t g0, int64_t g1) {
    int i0, j0, k0, i1, j1, k1;
    point_at(pg, g0, i0, j0, k0);
    point_at(pg, g1, i1, j1, k1);
    GridBox b;
    const bool row = k0 == k1 && (pg.tiled ? (j0 >> (6 - pg.tw_log)) == (j1 >> (6 - pg.tw_log)) : j0 == j1);
    b.xl = row ? (float)i0 : 0.0f;
    b.xh = row ? (float)i1 : (float)(pg.nx - 1);
    b.yl = k0 == k1 ? (float)j0 : 0.0f;
    b.yh = k0 == k1 ? (float)j1 : (float)(pg.nxy / pg.nx - 1);
    b.zl = -(float)k1;
    b.zh = -(float)k0;
    return b;
}

// wave w (points 64 w .. 64 w + 63) and group s (waves 64 s .. 64 s + 63)
__device__ __forceinline__ GridBox wave_box(const PointGeom& pg, int64_t w) {
    return range_box(pg, w * kWave, min(w * kWave + kWave - 1, pg.count - 1));
}
__device__ __forceinline__ GridBox group_box(const PointGeom& pg, int64_t s) {
    return range_box(pg, s * kWave * kWave, min((s + 1) * kWave * kWave - 1, pg.count - 1));
}

// T0 plus the box bounds of every track of one launch, below the still limit
__device__ __forceinline__ bool box_below(const EnvRec* __restrict__ e, int n, const GridBox& b, float T0,
                                          float rlim2) {
    float T = T0;
    for (int k = 0; k < n && T < kRestBelow; ++k) T += env_box_rise_bound(e[k], b, rlim2);
    return T < kRestBelow;
}

// One wave per launch and gpw groups of 64 waves: lane i < gpw tests the
// common box of one group; then the wave goes through its groups in turn,
// writing the 64 flags of a group (one per lane) from the group's test where
// it passed and from each wave's own box where it did not.  Far from the
// tracks a group passes as a whole, so most waves' boxes are never tested.
// gpw (1 .. 64) keeps enough waves in flight on small grids.
__global__ __launch_bounds__(kBlock) void still_flags_kernel(PointGeom pg, const EnvRec* __restrict__ env,
                                                            const int32_t* __restrict__ env_fc, int64_t nl,
                                                            int64_t n_waves, int gpw, float T0, float rlim2,
                                                            const GridBox* __restrict__ boxes,
                                                            uint8_t* __restrict__ flags) {
    const int64_t n_groups = wave_groups(n_waves);
    const int64_t blocks_per_launch = (n_groups + gpw - 1) / gpw;
    const int64_t gw = (int64_t)blockIdx.x * (kBlock / kWave) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (gw >= nl * blocks_per_launch) return;  // uniform per wave
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t l = gw / blocks_per_launch, s0 = (gw - l * blocks_per_launch) * gpw;
    const EnvRec* e = env + env_fc[2 * l];
    const int n = env_fc[2 * l + 1];
    const int64_t s = s0 + lane;
    bool pass = true;
    if (lane < gpw && s < n_groups) pass = box_below(e, n, boxes ? boxes[n_waves + s] : group_box(pg, s), T0, rlim2);
    const uint64_t passed = __ballot(pass);
    uint8_t* out = flags + l * n_waves;
    const int64_t s_end = min(n_groups, s0 + gpw);
    for (int64_t g = s0; g < s_end; ++g) {
        const int64_t w = g * kWave + lane;
        bool f = true;
        if (!((passed >> (g - s0)) & 1) && w < n_waves) f = box_below(e, n, boxes ? boxes[w] : wave_box(pg, w), T0, rlim2);
        if (w < n_waves) out[w] = f ? 1 : 0;
    }
}

hipError_t launch_still_flags(const PointGeom& pg, const EnvRec* env, const int32_t* env_fc, int64_t l0, int64_t nl,
                              int64_t n_waves, float T0, const GridBox* boxes, uint8_t* flags, hipStream_t st) {
    // groups per wave: 64, or fewer to keep about 8192 waves in flight
    const int64_t groups = wave_groups(n_waves) * nl;
    int gpw = 64;
    while (gpw > 1 && groups / gpw < 8192) gpw >>= 1;
    const int64_t waves = nl * ((wave_groups(n_waves) + gpw - 1) / gpw);
    if (waves <= 0) return hipSuccess;
    const int64_t wpb = kBlock / kWave;
    hipLaunchKernelGGL(still_flags_kernel, dim3((unsigned)((waves + wpb - 1) / wpb)), dim3(kBlock), 0, st, pg, env,
                       env_fc + 2 * l0, nl, n_waves, gpw, T0, envelope_radius2(pg), boxes, flags);
    return hipGetLastError();
}

// the box of each group of 64 waves from the waves' boxes (one lane per group)
__global__ __launch_bounds__(kBlock) void group_boxes_kernel(int64_t n_waves, GridBox* __restrict__ boxes) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= wave_groups(n_waves)) return;
    GridBox b = boxes[s * kWave];
    const int64_t w_end = min(n_waves, (s + 1) * kWave);
    for (int64_t w = s * kWave + 1; w < w_end; ++w) {
        const GridBox c = boxes[w];
        b.xl = fminf(b.xl, c.xl);
        b.xh = fmaxf(b.xh, c.xh);
        b.yl = fminf(b.yl, c.yl);
        b.yh = fmaxf(b.yh, c.yh);
        b.zl = fminf(b.zl, c.zl);
        b.zh = fmaxf(b.zh, c.zh);
    }
    boxes[n_waves + s] = b;
}

// one wave per wave of points: each lane decodes one point, the wave takes
// the least and greatest coordinates
__global__ __launch_bounds__(kBlock) void wave_boxes_kernel(PointGeom pg, int64_t n_waves,
                                                           GridBox* __restrict__ boxes) {
    const int64_t w = (int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
    if (w >= n_waves) return;  // uniform per wave
    const int64_t g = w * kWave + (threadIdx.x & (kWave - 1));
    int i0 = INT32_MAX, i1 = INT32_MIN, j0 = INT32_MAX, j1 = INT32_MIN, k0 = INT32_MAX, k1 = INT32_MIN;
    if (g < pg.count) {
        int gi, gj, gk;
        point_at(pg, g, gi, gj, gk);
        i0 = i1 = gi;
        j0 = j1 = gj;
        k0 = k1 = gk;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        i0 = min(i0, __shfl_xor(i0, o));
        i1 = max(i1, __shfl_xor(i1, o));
        j0 = min(j0, __shfl_xor(j0, o));
        j1 = max(j1, __shfl_xor(j1, o));
        k0 = min(k0, __shfl_xor(k0, o));
        k1 = max(k1, __shfl_xor(k1, o));
    }
    if ((threadIdx.x & (kWave - 1)) == 0)
        boxes[w] = GridBox{(float)i0, (float)i1, (float)j0, (float)j1, -(float)k1, -(float)k0};
}

hipError_t launch_wave_boxes(const PointGeom& pg, int64_t n_waves, GridBox* boxes, hipStream_t st) {
    if (n_waves <= 0) return hipSuccess;
    const int64_t blocks = (n_waves + kBlock / kWave - 1) / (kBlock / kWave);
    hipLaunchKernelGGL(wave_boxes_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, pg, n_waves, boxes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t groups = wave_groups(n_waves);
    hipLaunchKernelGGL(group_boxes_kernel, dim3((unsigned)((groups + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       n_waves, boxes);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fused K steps with the analytic temperature: one point per lane, its state
// held in registers (with compensated Euler accumulation); tab holds the
// K + 1 time points x W window slots of this launch.
// ---------------------------------------------------------------------------
// One launch of a wave on its register state (one point per lane, no
// tracked X~beta).  A wave whose points are all at rest and provably stay
// below the alpha_s -> beta end temperature at every time point of the
// launch is left as it is by every step (still).  Otherwise, a wave that no
// source of this launch reaches (every term of every track dropped at every
// time point) has T = T0 throughout (cold), and a cold wave whose first step
// changed nothing it stores stops there (frozen, see frozen_part).  The
// others take K explicit steps with the increments accumulated in (hi, lo)
// pairs.  a, m: the fractions as loaded in, and on return the fractions in
// memory after the launch (the loaded ones for a still or frozen wave, hi +
// lo otherwise); Tc: the temperature of the last correction (beta's sum
// rule).  Returns 0 (still), 1 (frozen) or 2 (stepped).  The fractions a
// still wave's beta and rest flag see are a + 0, m + 0.
template <int W>
__device__ __forceinline__ int plain_launch(const PointGeom& pg, const SrcRec* __restrict__ tab, const EnvSet& env,
                                            int64_t wv, int K, float dt, const ScanArgs& sa, bool act, int gi, int gj,
                                            int gk, float& a, float& m, float& Tc) {
    const float T0c = fminf(sa.T0, sa.Tclamp);
    const float rlim2 = envelope_radius2(pg);
    const bool tried = wave_may_rest(env, act, a, m, T0c);
    bool still = tried && (wave_box_below(env, wv) || wave_below(env.rec, env.n, act, gi, gj, gk, rlim2, T0c, kRestBelow));
    // an all-at-rest wave that is not below the limit everywhere is not cold either
    const bool cold = still || (!tried && wave_cold(env.rec, env.n, act, gi, gj, gk, rlim2));
    float Tn = cold ? T0c : scan_temperature<W>(tab, gi, gj, gk, sa.T0, sa.Tclamp, pg.r2min, pg.roff);
    Tc = Tn;
    float xeq_n = alpha_eq(Tn);
    // a cold wave whose points are all at rest at T0 is still as well
    still = still || (cold && T0c < Const<float>::TasEnd && __ballot(act && !rest_bits(a, m)) == 0);
    if (env.stats) count_wave(env, act, still, cold);
    if (still) return 0;
    // the waves that evaluate the temperature run the longest chains: they
    // issue first, and the other waves of their SIMD fill the gaps
    if (!cold) __builtin_amdgcn_s_setprio(3);
    const float a0 = a, m0 = m;
    float alo = 0.0f, mlo = 0.0f, Tblk = Tn;  // Tblk: sub-block start (wave counts only)
    bool frozen = false;
    for (int s = 0; s < K && !frozen; ++s) {
        const float Tn1 =
            cold ? T0c : scan_temperature<W>(tab + (s + 1) * W, gi, gj, gk, sa.T0, sa.Tclamp, pg.r2min, pg.roff);
        if (env.stats && !cold) {
            if (s % kStatBlock == 0) Tblk = Tn;
            if (s % kStatBlock == kStatBlock - 1) count_block(env, act, Tblk, Tn1);
        }
        const float xeq_n1 = alpha_eq(Tn1);
        explicit_step<true>(a, m, alo, mlo, Tn, xeq_n, Tn1, xeq_n1, dt, sa.rd);
        Tc = sa.rd.corr_prev ? Tn : Tn1;
        Tn = Tn1;
        xeq_n = xeq_n1;
        if (s == 0 && cold)
            frozen = __ballot(act && !(frozen_part(a0, a, alo, K) && frozen_part(m0, m, mlo, K))) == 0;
    }
    __builtin_amdgcn_s_setprio(0);
    if (frozen) {
        a = a0;
        m = m0;
        return 1;
    }
    a += alo;
    m += mlo;
    return 2;
}

// The points g0 + u kFusedBlock (u < PPT) of the calling lane; wv is the
// wave of the points for PPT = 1.  beta == nullptr: not written (inside a
// call only the last launch writes it; no kernel reads beta, it follows from
// the sum rule).  One point per lane without a tracked X~beta goes through
// plain_launch; the general form (PPT > 1, or TRACK) takes every launch
// certificate but the wave flags and the frozen stop.
template <int W, int PPT, bool TRACK>
__device__ __forceinline__ void fused_plain_body(const PointGeom& pg, const SrcRec* __restrict__ tab,
                                                 const EnvSet& env, int K, float dt, const ScanArgs& sa,
                                                 float* __restrict__ beta, float* __restrict__ as,
                                                 float* __restrict__ am, double* __restrict__ xbv, int64_t g0,
                                                 int64_t wv) {
    if constexpr (PPT == 1 && !TRACK) {
        bool act = g0 < pg.count;
        int gi, gj, gk;
        const int64_t local = point_at(pg, act ? g0 : 0, gi, gj, gk);
        act = act && gk >= pg.k0;
        float a = act ? as[local] : 0.0f, m = act ? am[local] : 0.0f, Tc;
        const int r = plain_launch<W>(pg, tab, env, wv, K, dt, sa, act, gi, gj, gk, a, m, Tc);
        const float af = r == 0 ? a + 0.0f : a, mf = r == 0 ? m + 0.0f : m;
        if (act) {
            if (r == 2) {  // a still or frozen wave's fractions are those in memory
                as[local] = af;
                am[local] = mf;
            }
            if (beta) beta[local] = solid_fraction(Tc) - af - mf;
        }
        record_rest(env, wv, act, af, mf);
        return;
    } else {
        const float T0c = fminf(sa.T0, sa.Tclamp);
        int64_t local[PPT];
        int gi[PPT], gj[PPT], gk[PPT];
        bool act[PPT];
        float a[PPT], m[PPT], alo[PPT], mlo[PPT], Tn[PPT], xeq_n[PPT], Tc[PPT];
        double xb[PPT];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int64_t g = g0 + u * kFusedBlock;
            act[u] = g < pg.count;
            local[u] = point_at(pg, act[u] ? g : 0, gi[u], gj[u], gk[u]);
            act[u] = act[u] && gk[u] >= pg.k0;
            a[u] = act[u] ? as[local[u]] : 0.0f;
            m[u] = act[u] ? am[local[u]] : 0.0f;
            xb[u] = (TRACK && act[u]) ? track_check(xbv[local[u]], a[u], m[u]) : track_none();
            alo[u] = 0.0f;
            mlo[u] = 0.0f;
        }
        // still and cold waves as in plain_launch
        bool cold[PPT], still[PPT];
        const float rlim2 = envelope_radius2(pg);
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const bool tried = wave_may_rest(env, act[u], a[u], m[u], T0c);
            still[u] = tried && wave_below(env.rec, env.n, act[u], gi[u], gj[u], gk[u], rlim2, T0c, kRestBelow);
            cold[u] = still[u] || (!tried && wave_cold(env.rec, env.n, act[u], gi[u], gj[u], gk[u], rlim2));
            Tn[u] = cold[u] ? T0c : scan_temperature<W>(tab, gi[u], gj[u], gk[u], sa.T0, sa.Tclamp, pg.r2min, pg.roff);
            Tc[u] = Tn[u];
            xeq_n[u] = alpha_eq(Tn[u]);
            still[u] = still[u] || (cold[u] && T0c < Const<float>::TasEnd && __ballot(act[u] && !rest_bits(a[u], m[u])) == 0);
            if (TRACK && still[u]) xb[u] = track_none();
            if (env.stats) count_wave(env, act[u], still[u], cold[u]);
        }
        float Tblk[PPT];
        for (int s = 0; s < K; ++s) {
#pragma unroll
            for (int u = 0; u < PPT; ++u) {
                if (still[u]) continue;
                const float Tn1 = cold[u] ? T0c
                                          : scan_temperature<W>(tab + (s + 1) * W, gi[u], gj[u], gk[u], sa.T0, sa.Tclamp,
                                                                pg.r2min, pg.roff);
                if (env.stats && !cold[u]) {
                    if (s % kStatBlock == 0) Tblk[u] = Tn[u];
                    if (s % kStatBlock == kStatBlock - 1) count_block(env, act[u], Tblk[u], Tn1);
                }
                const float xeq_n1 = alpha_eq(Tn1);
                if (TRACK)
                    explicit_step_tracked<true>(a[u], m[u], alo[u], mlo[u], xb[u], Tn[u], xeq_n[u], Tn1, xeq_n1, dt,
                                                sa.rd);
                else
                    explicit_step<true>(a[u], m[u], alo[u], mlo[u], Tn[u], xeq_n[u], Tn1, xeq_n1, dt, sa.rd);
                Tc[u] = sa.rd.corr_prev ? Tn[u] : Tn1;
                Tn[u] = Tn1;
                xeq_n[u] = xeq_n1;
            }
        }
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            if (!act[u]) continue;
            const float af = a[u] + alo[u], mf = m[u] + mlo[u];
            if (!still[u]) {  // a still wave's fractions are those in memory
                as[local[u]] = af;
                am[local[u]] = mf;
            }
            if (TRACK) xbv[local[u]] = xb[u];
            if (beta) beta[local[u]] = solid_fraction(Tc[u]) - af - mf;
        }
    }
}

// PPT points per lane, kFusedBlock apart (coalesced), advanced together for ILP
template <int W, int PPT, bool TRACK>
__global__ __launch_bounds__(kFusedBlock) void fused_plain_kernel(PointGeom pg, const SrcRec* __restrict__ tab,
                                                                  EnvSet env, int K, float dt, ScanArgs sa,
                                                                  float* __restrict__ beta, float* __restrict__ as,
                                                                  float* __restrict__ am, double* __restrict__ xbv) {
    const int64_t wv = fused_wave();
    if (PPT == 1 && !TRACK && wave_flag_still(env, wv)) {
        still_wave_beta(pg, fminf(sa.T0, sa.Tclamp), beta, (int64_t)blockIdx.x * kFusedBlock + threadIdx.x);
        if (env.stats && (threadIdx.x & (kWave - 1)) == 0) atomicAdd(env.stats + kStatFlagged, 1ull);
        return;
    }
    fused_plain_body<W, PPT, TRACK>(pg, tab, env, K, dt, sa, beta, as, am, xbv,
                                    (int64_t)blockIdx.x * kFusedBlock * PPT + threadIdx.x, wv);
}

// One implicit launch of a wave on its register state (one point per lane,
// no tracked X~beta), as plain_launch: still and cold waves as there, and a
// cold wave whose first step changed nothing it stores stops there (see
// frozen_part): with the high parts unchanged after every substep, each
// substep's iteration starts from the same state, converges at its first
// iterate with a zero residual and adds the same increments to the low
// parts; a first step with an unconverged substep does not stop, so that
// the count stays exact.  Adds the lane's unconverged substeps to bad.
template <int W>
__device__ __forceinline__ int implicit_launch(const PointGeom& pg, const SrcRec* __restrict__ tab, const EnvSet& env,
                                               int64_t wv, int K, float h, int n_sub, int max_iter, const ScanArgs& sa,
                                               bool act, int gi, int gj, int gk, float& a, float& m, float& Tc,
                                               int& bad) {
    const float T0c = fminf(sa.T0, sa.Tclamp);
    const float rlim2 = envelope_radius2(pg);
    const bool tried = wave_may_rest(env, act, a, m, T0c);
    bool still = tried && (wave_box_below(env, wv) || wave_below(env.rec, env.n, act, gi, gj, gk, rlim2, T0c, kRestBelow));
    const bool cold = still || (!tried && wave_cold(env.rec, env.n, act, gi, gj, gk, rlim2));
    float Tn = cold ? T0c : scan_temperature<W>(tab, gi, gj, gk, sa.T0, sa.Tclamp, pg.r2min, pg.roff);
    Tc = Tn;
    still = still || (cold && T0c < Const<float>::TasEnd && __ballot(act && !rest_bits(a, m)) == 0);
    if (env.stats) count_wave(env, act, still, cold);
    if (still) return 0;
    if (!cold) __builtin_amdgcn_s_setprio(3);  // as in plain_launch
    const float inv = 1.0f / (float)n_sub;
    const float a0 = a, m0 = m;
    float alo = 0.0f, mlo = 0.0f, b = 0.0f;
    int lbad = 0;
    bool frozen = false;
    for (int s = 0; s < K && !frozen; ++s) {
        const float Tn1 =
            cold ? T0c : scan_temperature<W>(tab + (s + 1) * W, gi, gj, gk, sa.T0, sa.Tclamp, pg.r2min, pg.roff);
        float Ta = Tn;
        bool same = true;
        for (int k = 0; k < n_sub; ++k) {
            const float Tb = (k + 1 == n_sub) ? Tn1 : fmaf(Tn1 - Tn, (float)(k + 1) * inv, Tn);
            if (implicit_step<true>(a, m, alo, mlo, b, Ta, Tb, h, max_iter, sa.rd.mart_assign) < 0) ++lbad;
            same = same && __float_as_uint(a) == __float_as_uint(a0) && __float_as_uint(m) == __float_as_uint(m0);
            Ta = Tb;
        }
        Tn = Tn1;
        if (s == 0 && cold)
            frozen = __ballot(act && !(same && lbad == 0 && frozen_part(a0, a, alo, K) && frozen_part(m0, m, mlo, K))) == 0;
    }
    __builtin_amdgcn_s_setprio(0);
    Tc = Tn;
    if (act) bad += lbad;
    if (frozen) {
        a = a0;
        m = m0;
        return 1;
    }
    a += alo;
    m += mlo;
    return 2;
}

// the lanes' counts of unconverged substeps, summed over the wave and added
// to the context's count (by every lane, lane 0 with the sum)
__device__ __forceinline__ void add_unconverged(unsigned long long* unconverged, int bad) {
    int total = bad;
    for (int o = 32; o > 0; o >>= 1) total += __shfl_xor(total, o);
    if (total) atomicAdd(unconverged, (threadIdx.x & (kWave - 1)) == 0 ? (unsigned long long)total : 0ull);
}

// workgroup of the list passes (sixteen waves; see candidates_kernel)
constexpr int kListBlock = 1024;

// The waves of a chunk of launches l0 .. l0 + nl - 1 that the call kernel
// takes: one wave per wave of points finds whether it is at rest (from its
// state in the first chunk of a call, from its rest flag after) and loads its
// still flags for the chunk (lane i: launch l0 + i, 64 at a time).  A wave
// at rest that the box pre-pass bounds below the still limit in every launch
// of the chunk is still throughout it: its rest flag is set and, if the
// chunk ends the call, beta written.  The others are listed (one atomic per
// workgroup of 16 waves) in cand[0 .. counts[0]).
__global__ __launch_bounds__(kListBlock) void chunk_list_kernel(
    PointGeom pg, const uint8_t* __restrict__ below, uint8_t* __restrict__ rest, int64_t n_waves, int64_t l0,
    int64_t nl, float T0c, float* __restrict__ beta, const float* __restrict__ as, const float* __restrict__ am,
    uint32_t* __restrict__ cand, unsigned* __restrict__ counts, unsigned long long* __restrict__ stats) {
    __shared__ unsigned wave_n[kListBlock / kWave + 1];
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int64_t w = (int64_t)blockIdx.x * (kListBlock / kWave) + wib;
    const int lane = threadIdx.x & (kWave - 1);
    const bool in = w < n_waves;  // uniform per wave
    bool still = false;
    if (in) {
        const int64_t g = w * kWave + lane;
        bool act = g < pg.count;
        int gi, gj, gk;
        const int64_t local = point_at(pg, act ? g : 0, gi, gj, gk);
        act = act && gk >= pg.k0;
        // the first 64 launches' flags are loaded with the state, not after it
        // (lanes past nl load launch nl - 1's flag and ignore it; nl >= 1)
        const uint8_t f0 = below[min((int64_t)lane, nl - 1) * n_waves + w];
        float a = 0.0f, m = 0.0f;
        uint8_t r = 0;
        if (l0 == 0) {  // (below implies T0 under the still limit)
            a = act ? as[local] : 0.0f;
            m = act ? am[local] : 0.0f;
        } else {
            r = rest[w];
        }
        const bool at_rest = l0 == 0 ? __ballot(act && !rest_bits(a, m)) == 0 : r != 0;
        still = at_rest && __ballot(lane < nl && f0 == 0) == 0;
        for (int64_t i0 = kWave; i0 < nl && still; i0 += kWave)
            still = __ballot(i0 + lane < nl && below[(i0 + lane) * n_waves + w] == 0) == 0;
        if (still) {
            if (act && beta) beta[local] = solid_fraction(T0c) - kXmax - 0.0f;
            if (stats) atomicAdd(stats + kStatFlagged, lane == 0 ? (unsigned long long)nl : 0ull);
            rest[w] = 1;  // (the same byte from every lane)
        }
    }
    if (lane == 0) wave_n[wib] = (in && !still) ? 1u : 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned total = 0;
        for (int i = 0; i < kListBlock / kWave; ++i) {
            const unsigned c = wave_n[i];
            wave_n[i] = total;
            total += c;
        }
        wave_n[kListBlock / kWave] = total ? atomicAdd(counts, total) : 0u;
    }
    __syncthreads();
    if (in && !still && lane == 0) cand[wave_n[kListBlock / kWave] + wave_n[wib]] = (uint32_t)w;
}

// ---------------------------------------------------------------------------
// A fused PLAIN call, or a chunk of its launches, in one persistent kernel:
// each wave of the grid takes waves of points from a shared counter, loads
// one once, runs every launch of the chunk on its registers (plain_launch;
// a launch that the wave flags say is still costs one byte) and stores it
// once.  The waves of points do not depend on each other, so no launch waits
// for the whole grid to finish the one before: the few waves near the
// tracks, which run chains of K dependent steps launch after launch, share
// the GPU with the rest of the call instead of ending every launch alone.
// What each point computes is what the launch-by-launch form computes, bit
// for bit: a launch starts from the fractions the previous one left in
// memory (hi + lo), and a still or frozen launch leaves them as they were.
// Wave flags: below (the chunk's still flags, [l - l0][w]), rest (per wave,
// at rest after the last launch that took its steps: read from the second
// chunk, written at the end of each).
// ---------------------------------------------------------------------------
// grid waves of the persistent call kernels: eight per SIMD (their registers
// let seven stay resident; the rest start as the first workgroups end and
// take what is left of the list)
constexpr int kCallWaves = 256 * 4 * 8;

// The loop of a call kernel: launch(es, w, tab_l, Kl, act, gi, gj, gk, a, m,
// Tc) runs one launch on a wave's register state as plain_launch does.
template <class Launch>
__device__ __forceinline__ void fused_call(const PointGeom& pg, const SrcRec* __restrict__ tab,
                                           const EnvRec* __restrict__ env, const int32_t* __restrict__ env_fc,
                                           const uint8_t* __restrict__ below, uint8_t* __restrict__ rest,
                                           int64_t n_waves, int64_t l0, int64_t nl, int K, int64_t n_steps, int W,
                                           float T0c, float* __restrict__ beta, float* __restrict__ as,
                                           float* __restrict__ am, const uint32_t* __restrict__ cand,
                                           const unsigned* __restrict__ cand_n, unsigned* __restrict__ next,
                                           unsigned long long* __restrict__ stats, Launch launch) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t n_list = *cand_n;
    // No branch on the lane inside this loop: every lane takes part in the
    // atomic (lane 0 adds 1, the others 0) and lane 0's old value is the
    // wave's, and the per-wave stores are made by all lanes.  (A lane-0
    // branch at the top and another at the bottom of the body let the
    // compiler send lane 0 round the loop alone, so that the other lanes
    // read the wave number from an inactive lane and never left.)
    for (;;) {
        const unsigned ei = atomicAdd(next, lane == 0 ? 1u : 0u);
        const int64_t e = (int64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)ei);
        if (e >= n_list) return;  // uniform per wave: every wave ends once the counter passes the list
        const int64_t w = (int64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)cand[e]);
        const int64_t g = w * kWave + lane;
        bool act = g < pg.count;
        int gi, gj, gk;
        const int64_t local = point_at(pg, act ? g : 0, gi, gj, gk);
        act = act && gk >= pg.k0;
        float a = act ? as[local] : 0.0f, m = act ? am[local] : 0.0f;
        float af = a, mf = m, Tc = T0c;
        // at rest: from the state for the first launch of a call (below implies T0 under the limit)
        bool rest_w = l0 == 0 ? __ballot(act && !rest_bits(a, m)) == 0 : rest[w] != 0;
        bool changed = false, flagged = false;
        uint64_t bm = 0;  // the wave's still flags for launches lb .. lb + 63, one bit each
        int64_t lb = l0 - kWave;
        for (int64_t l = l0; l < l0 + nl; ++l) {
            const uint8_t* bl = below + (l - l0) * n_waves;
            if (l - lb >= kWave) {  // (uniform) lane i loads launch l + i's flag
                lb = l;
                bm = __ballot(l + lane < l0 + nl && below[(l - l0 + lane) * n_waves + w] != 0);
            }
            flagged = rest_w && ((bm >> (l - lb)) & 1);
            if (flagged) {  // still by its flags: nothing read, nothing changes
                if (stats) atomicAdd(stats + kStatFlagged, lane == 0 ? 1ull : 0ull);
                continue;
            }
            const int64_t s0 = l * K;
            const int Kl = (int)min((int64_t)K, n_steps - s0);
            const EnvSet es{env + env_fc[2 * l], env_fc[2 * l + 1], bl, nullptr, n_waves, 0, stats,
                            nullptr, nullptr, nullptr};
            const int r = launch(es, w, tab + s0 * W, Kl, act, gi, gj, gk, a, m, Tc);
            af = r == 0 ? a + 0.0f : a;
            mf = r == 0 ? m + 0.0f : m;
            changed = changed || r == 2;
            rest_w = __ballot(act && !rest_bits(af, mf)) == 0;
        }
        if (act) {
            if (changed) {
                as[local] = a;
                am[local] = m;
            }
            if (beta) beta[local] = flagged ? solid_fraction(T0c) - kXmax - 0.0f : solid_fraction(Tc) - af - mf;
        }
        rest[w] = rest_w ? 1 : 0;  // (the same byte from every lane)
    }
}

template <int W>
__global__ __launch_bounds__(kCallBlock) void fused_plain_call_kernel(
    PointGeom pg, const SrcRec* __restrict__ tab, const EnvRec* __restrict__ env, const int32_t* __restrict__ env_fc,
    const uint8_t* __restrict__ below, uint8_t* __restrict__ rest, int64_t n_waves, int64_t l0, int64_t nl, int K,
    int64_t n_steps, float dt, ScanArgs sa, float* __restrict__ beta, float* __restrict__ as, float* __restrict__ am,
    const uint32_t* __restrict__ cand, const unsigned* __restrict__ cand_n, unsigned* __restrict__ next,
    unsigned long long* __restrict__ stats) {
    fused_call(pg, tab, env, env_fc, below, rest, n_waves, l0, nl, K, n_steps, W, fminf(sa.T0, sa.Tclamp), beta, as,
               am, cand, cand_n, next, stats,
               [&](const EnvSet& es, int64_t w, const SrcRec* t, int Kl, bool act, int gi, int gj, int gk, float& a,
                   float& m, float& Tc) {
                   return plain_launch<W>(pg, t, es, w, Kl, dt, sa, act, gi, gj, gk, a, m, Tc);
               });
}

// the list pass of a chunk (counts cleared first)
hipError_t launch_chunk_list(const PointGeom& pg, const uint8_t* below, uint8_t* rest, int64_t n_waves, int64_t l0,
                             int64_t nl, float T0c, float* beta, const float* as, const float* am, uint32_t* cand,
                             unsigned* counts, unsigned long long* stats, hipStream_t st) {
    hipError_t e = launch_clear_counts(counts, st);
    if (e != hipSuccess || n_waves <= 0 || nl <= 0) return e;
    const int64_t lpb = kListBlock / kWave;
    hipLaunchKernelGGL(chunk_list_kernel, dim3((unsigned)((n_waves + lpb - 1) / lpb)), dim3(kListBlock), 0, st, pg,
                       below, rest, n_waves, l0, nl, T0c, beta, as, am, cand, counts, stats);
    return hipGetLastError();
}

dim3 call_grid(int64_t n_waves) {
    const int64_t wpb = kCallBlock / kWave;
    const int64_t waves = n_waves < kCallWaves ? n_waves : kCallWaves;
    return dim3((unsigned)((waves + wpb - 1) / wpb));
}

hipError_t launch_fused_plain_call(const PointGeom& pg, int W, const SrcRec* tab, const EnvRec* env,
                                   const int32_t* env_fc, const uint8_t* below, uint8_t* rest, int64_t n_waves,
                                   int64_t l0, int64_t nl, int K, int64_t n_steps, float dt, ScanArgs sa, float* beta,
                                   float* as, float* am, uint32_t* cand, unsigned* counts,
                                   unsigned long long* stats, hipStream_t st) {
    if (n_waves <= 0 || nl <= 0) return hipSuccess;
    hipError_t e = launch_chunk_list(pg, below, rest, n_waves, l0, nl, fminf(sa.T0, sa.Tclamp), beta, as, am, cand,
                                     counts, stats, st);
    if (e != hipSuccess) return e;
    const dim3 grid = call_grid(n_waves), block(kCallBlock);
    switch (W) {
        case 1: hipLaunchKernelGGL(fused_plain_call_kernel<1>, grid, block, 0, st, pg, tab, env, env_fc, below, rest, n_waves, l0, nl, K, n_steps, dt, sa, beta, as, am, cand, counts, counts + 1, stats); break;
        case 2: hipLaunchKernelGGL(fused_plain_call_kernel<2>, grid, block, 0, st, pg, tab, env, env_fc, below, rest, n_waves, l0, nl, K, n_steps, dt, sa, beta, as, am, cand, counts, counts + 1, stats); break;
        case 3: hipLaunchKernelGGL(fused_plain_call_kernel<3>, grid, block, 0, st, pg, tab, env, env_fc, below, rest, n_waves, l0, nl, K, n_steps, dt, sa, beta, as, am, cand, counts, counts + 1, stats); break;
        case 4: hipLaunchKernelGGL(fused_plain_call_kernel<4>, grid, block, 0, st, pg, tab, env, env_fc, below, rest, n_waves, l0, nl, K, n_steps, dt, sa, beta, as, am, cand, counts, counts + 1, stats); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// One wave per 64 waves of a slot launch: the waves that are not still by
// their flags go to the launch's list, the still ones write beta in the
// last launch of a call.  A workgroup of 16 waves takes its places in the
// list with one atomic (all workgroups add to the same count, so atomics per
// wave would queue up: 16.8 us per launch on a 1M-wave grid).

__global__ __launch_bounds__(kListBlock) void candidates_kernel(PointGeom pg, EnvSet env, float T0c,
                                                               float* __restrict__ beta) {
    __shared__ unsigned wave_n[kListBlock / kWave + 1];
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int64_t gw = (int64_t)blockIdx.x * (kListBlock / kWave) + wib;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = gw * kWave + lane;
    const bool in = w < env.n_waves;
    const bool still = in && env.below[w] && env.rest[w];
    const uint64_t todo = __ballot(in && !still);
    uint64_t quiet = beta ? __ballot(still) : 0;
    if (env.stats) {
        const int nq = __popcll(__ballot(still));
        if (nq && lane == 0) atomicAdd(env.stats + kStatFlagged, (unsigned long long)nq);
    }
    if (lane == 0) wave_n[wib] = (unsigned)__popcll(todo);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned total = 0;
        for (int i = 0; i < kListBlock / kWave; ++i) {
            const unsigned c = wave_n[i];
            wave_n[i] = total;
            total += c;
        }
        wave_n[kListBlock / kWave] = total ? atomicAdd(env.cand_n, total) : 0u;
    }
    __syncthreads();
    const unsigned base = wave_n[kListBlock / kWave] + wave_n[wib];
    if (in && !still) env.cand[base + __popcll(todo & ((1ull << lane) - 1))] = (uint32_t)w;
    while (quiet) {
        const int i = __builtin_ctzll(quiet);
        quiet &= quiet - 1;
        still_wave_beta(pg, T0c, beta, (gw * kWave + i) * kWave + lane);
    }
}

// The first launch of a call, which has no rest flags yet: one wave per
// wave of points reads its state; a wave at rest that the box pre-pass
// bounds below the still limit is still (its rest flag is set and, in a
// one-launch call, beta written), the others go to the list (one atomic per
// workgroup of 16 waves).
__global__ __launch_bounds__(kListBlock) void first_candidates_kernel(PointGeom pg, EnvSet env, float T0c,
                                                                     float* __restrict__ beta,
                                                                     const float* __restrict__ as,
                                                                     const float* __restrict__ am) {
    __shared__ unsigned wave_n[kListBlock / kWave + 1];
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int64_t w = (int64_t)blockIdx.x * (kListBlock / kWave) + wib;
    const int lane = threadIdx.x & (kWave - 1);
    const bool in = w < env.n_waves;  // uniform per wave
    bool still = false;
    if (in) {
        const int64_t g = w * kWave + lane;
        bool act = g < pg.count;
        int gi, gj, gk;
        const int64_t local = point_at(pg, act ? g : 0, gi, gj, gk);
        act = act && gk >= pg.k0;
        const float a = act ? as[local] : 0.0f, m = act ? am[local] : 0.0f;
        still = env.below[w] && wave_may_rest(env, act, a, m, T0c);
        if (still) {
            if (act && beta) beta[local] = solid_fraction(T0c) - a - m;
            if (env.stats) count_wave(env, act, true, true);
            if (lane == 0) env.rest[w] = 1;
        }
    }
    if (lane == 0) wave_n[wib] = (in && !still) ? 1u : 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned total = 0;
        for (int i = 0; i < kListBlock / kWave; ++i) {
            const unsigned c = wave_n[i];
            wave_n[i] = total;
            total += c;
        }
        wave_n[kListBlock / kWave] = total ? atomicAdd(env.cand_n, total) : 0u;
    }
    __syncthreads();
    if (in && !still && lane == 0) env.cand[wave_n[kListBlock / kWave] + wave_n[wib]] = (uint32_t)w;
}

hipError_t launch_first_candidates(const PointGeom& pg, const EnvSet& env, float T0c, float* beta, const float* as,
                                   const float* am, hipStream_t st) {
    const int64_t wpb = kListBlock / kWave;
    if (env.n_waves <= 0) return hipSuccess;
    hipLaunchKernelGGL(first_candidates_kernel, dim3((unsigned)((env.n_waves + wpb - 1) / wpb)), dim3(kListBlock), 0,
                       st, pg, env, T0c, beta, as, am);
    return hipGetLastError();
}

hipError_t launch_candidates(const PointGeom& pg, const EnvSet& env, float T0c, float* beta, hipStream_t st) {
    const int64_t waves = (env.n_waves + kWave - 1) / kWave, wpb = kListBlock / kWave;
    if (waves <= 0) return hipSuccess;
    hipLaunchKernelGGL(candidates_kernel, dim3((unsigned)((waves + wpb - 1) / wpb)), dim3(kListBlock), 0, st, pg,
                       env, T0c, beta);
    return hipGetLastError();
}

__global__ void clear_counts_kernel(unsigned* c) {
    if (threadIdx.x < 2) c[threadIdx.x] = 0u;
}

hipError_t launch_clear_counts(unsigned* counts, hipStream_t st) {
    hipLaunchKernelGGL(clear_counts_kernel, dim3(1), dim3(64), 0, st, counts);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fused K steps with the implicit scheme: as the plain fused kernel, with the
// Crank-Nicolson fixed-point step at every step (n_sub equal substeps of
// length h when the step exceeds the substep limit, T linear between the
// analytic step-end values), with compensated accumulation of the increments
// inside a launch as in the plain fused kernel.
// ---------------------------------------------------------------------------
template <int W, bool TRACK>
__device__ __forceinline__ void fused_implicit_body(const PointGeom& pg, const SrcRec* __restrict__ tab,
                                                    const EnvSet& env, int K, float h, int n_sub, int max_iter,
                                                    const ScanArgs& sa, float* __restrict__ beta,
                                                    float* __restrict__ as, float* __restrict__ am,
                                                    double* __restrict__ xbv,
                                                    unsigned long long* __restrict__ unconverged, int64_t g,
                                                    int64_t wv) {
    const float T0c = fminf(sa.T0, sa.Tclamp);
    bool act = g < pg.count;
    int gi, gj, gk;
    const int64_t local = point_at(pg, act ? g : 0, gi, gj, gk);
    act = act && gk >= pg.k0;
    float a = act ? as[local] : 0.0f, m = act ? am[local] : 0.0f;
    int bad = 0;
    if constexpr (!TRACK) {
        float Tc;
        const int r = implicit_launch<W>(pg, tab, env, wv, K, h, n_sub, max_iter, sa, act, gi, gj, gk, a, m, Tc, bad);
        const float af = r == 0 ? a + 0.0f : a, mf = r == 0 ? m + 0.0f : m;
        if (act) {
            if (r == 2) {  // a still or frozen wave's fractions are those in memory
                as[local] = af;
                am[local] = mf;
            }
            if (beta) beta[local] = solid_fraction(Tc) - af - mf;
        }
        record_rest(env, wv, act, af, mf);
    } else {
        float b = 0.0f, alo = 0.0f, mlo = 0.0f;
        double xb = act ? track_check(xbv[local], a, m) : track_none();
        // still and cold waves as in plain_launch (without the wave flags)
        const float rlim2 = envelope_radius2(pg);
        const bool tried = wave_may_rest(env, act, a, m, T0c);
        bool still = tried && wave_below(env.rec, env.n, act, gi, gj, gk, rlim2, T0c, kRestBelow);
        const bool cold = still || (!tried && wave_cold(env.rec, env.n, act, gi, gj, gk, rlim2));
        float Tn = cold ? T0c : scan_temperature<W>(tab, gi, gj, gk, sa.T0, sa.Tclamp, pg.r2min, pg.roff);
        const float inv = 1.0f / (float)n_sub;
        still = still || (cold && T0c < Const<float>::TasEnd && __ballot(act && !rest_bits(a, m)) == 0);
        if (still) xb = track_none();
        if (env.stats) count_wave(env, act, still, cold);
        for (int s = 0; s < K && !still; ++s) {
            const float Tn1 =
                cold ? T0c : scan_temperature<W>(tab + (s + 1) * W, gi, gj, gk, sa.T0, sa.Tclamp, pg.r2min, pg.roff);
            float Ta = Tn;
            for (int k = 0; k < n_sub; ++k) {
                const float Tb = (k + 1 == n_sub) ? Tn1 : fmaf(Tn1 - Tn, (float)(k + 1) * inv, Tn);
                if (implicit_step_tracked<true>(a, m, alo, mlo, xb, b, Ta, Tb, h, max_iter, sa.rd.mart_assign) < 0)
                    ++bad;
                Ta = Tb;
            }
            Tn = Tn1;
        }
        if (act) {
            a += alo;
            m += mlo;
            if (!still) {  // a still wave's fractions are those in memory
                as[local] = a;
                am[local] = m;
            }
            if (beta) beta[local] = solid_fraction(Tn) - a - m;
            xbv[local] = xb;
        }
        if (!act) bad = 0;
    }
    add_unconverged(unconverged, bad);
}

template <int W, bool TRACK>
__global__ __launch_bounds__(kFusedBlock) void fused_implicit_kernel(PointGeom pg, const SrcRec* __restrict__ tab,
                                                                     EnvSet env, int K, float h, int n_sub,
                                                                     int max_iter, ScanArgs sa,
                                                                     float* __restrict__ beta, float* __restrict__ as,
                                                                     float* __restrict__ am, double* __restrict__ xbv,
                                                                     unsigned long long* __restrict__ unconverged) {
    const int64_t wv = fused_wave();
    const int64_t g = (int64_t)blockIdx.x * kFusedBlock + threadIdx.x;
    if (!TRACK && wave_flag_still(env, wv)) {  // see fused_plain_kernel
        still_wave_beta(pg, fminf(sa.T0, sa.Tclamp), beta, g);
        if (env.stats && (threadIdx.x & (kWave - 1)) == 0) atomicAdd(env.stats + kStatFlagged, 1ull);
        return;
    }
    fused_implicit_body<W, TRACK>(pg, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, xbv, unconverged, g, wv);
}

template <bool TRACK>
static hipError_t fused_implicit_w(const PointGeom& pg, int W, const SrcRec* tab, EnvSet env, int K, float h,
                                   int n_sub, int max_iter, ScanArgs sa, float* beta, float* as, float* am, double* xb,
                                   unsigned long long* unconverged, hipStream_t st) {
    const dim3 grid((unsigned)((pg.count + kFusedBlock - 1) / kFusedBlock)), block(kFusedBlock);
    switch (W) {
        case 1: hipLaunchKernelGGL((fused_implicit_kernel<1, TRACK>), grid, block, 0, st, pg, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, xb, unconverged); break;
        case 2: hipLaunchKernelGGL((fused_implicit_kernel<2, TRACK>), grid, block, 0, st, pg, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, xb, unconverged); break;
        case 3: hipLaunchKernelGGL((fused_implicit_kernel<3, TRACK>), grid, block, 0, st, pg, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, xb, unconverged); break;
        case 4: hipLaunchKernelGGL((fused_implicit_kernel<4, TRACK>), grid, block, 0, st, pg, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, xb, unconverged); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int W, int BS>
__global__ __launch_bounds__(BS) void fused_implicit_slots_kernel(
    PointGeom pg, const SrcRec* __restrict__ tab, EnvSet env, int K, float h, int n_sub, int max_iter, ScanArgs sa,
    float* __restrict__ beta, float* __restrict__ as, float* __restrict__ am,
    unsigned long long* __restrict__ unconverged) {
    const int lane = threadIdx.x & (kWave - 1);
    fused_slots<BS>(env, [&](int64_t w) {
        fused_implicit_body<W, false>(pg, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, nullptr, unconverged,
                                      w * kWave + lane, w);
    });
}

hipError_t launch_fused_implicit(const PointGeom& pg, int W, const SrcRec* tab, EnvSet env, int K, float h, int n_sub,
                                 int max_iter, ScanArgs sa, float* beta, float* as, float* am, double* xb,
                                 unsigned long long* unconverged, hipStream_t st) {
    if (pg.count <= 0) return hipSuccess;
    if (!xb && env.below && env.cand) {
        switch (W) {
            case 1: LAUNCH_SLOTS(fused_implicit_slots_kernel, 1, env.n_waves, slots_per_wave(env.n_waves), st, pg, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, unconverged); break;
            case 2: LAUNCH_SLOTS(fused_implicit_slots_kernel, 2, env.n_waves, slots_per_wave(env.n_waves), st, pg, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, unconverged); break;
            case 3: LAUNCH_SLOTS(fused_implicit_slots_kernel, 3, env.n_waves, slots_per_wave(env.n_waves), st, pg, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, unconverged); break;
            case 4: LAUNCH_SLOTS(fused_implicit_slots_kernel, 4, env.n_waves, slots_per_wave(env.n_waves), st, pg, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, unconverged); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    return xb ? fused_implicit_w<true>(pg, W, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, xb, unconverged, st)
              : fused_implicit_w<false>(pg, W, tab, env, K, h, n_sub, max_iter, sa, beta, as, am, xb, unconverged, st);
}

hipError_t launch_temperature(const PointGeom& pg, int W, const SrcRec* rec, ScanArgs sa, float* T,
                              hipStream_t st) {
    if (pg.count <= 0) return hipSuccess;
    const dim3 grid((unsigned)((pg.count + kBlock - 1) / kBlock)), block(kBlock);
    switch (W) {
        case 1: hipLaunchKernelGGL(temperature_kernel<1>, grid, block, 0, st, pg, rec, sa, T); break;
        case 2: hipLaunchKernelGGL(temperature_kernel<2>, grid, block, 0, st, pg, rec, sa, T); break;
        case 3: hipLaunchKernelGGL(temperature_kernel<3>, grid, block, 0, st, pg, rec, sa, T); break;
        case 4: hipLaunchKernelGGL(temperature_kernel<4>, grid, block, 0, st, pg, rec, sa, T); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

constexpr int kFusedPPT = FUSED_PPT;

template <bool TRACK>
static hipError_t fused_plain_w(const PointGeom& pg, int W, const SrcRec* tab, EnvSet env, int K, float dt,
                                ScanArgs sa, float* beta, float* as, float* am, double* xb, hipStream_t st) {
    const dim3 grid((unsigned)((pg.count + kFusedBlock * kFusedPPT - 1) / (kFusedBlock * kFusedPPT))), block(kFusedBlock);
    switch (W) {
        case 1: hipLaunchKernelGGL((fused_plain_kernel<1, kFusedPPT, TRACK>), grid, block, 0, st, pg, tab, env, K, dt, sa, beta, as, am, xb); break;
        case 2: hipLaunchKernelGGL((fused_plain_kernel<2, kFusedPPT, TRACK>), grid, block, 0, st, pg, tab, env, K, dt, sa, beta, as, am, xb); break;
        case 3: hipLaunchKernelGGL((fused_plain_kernel<3, kFusedPPT, TRACK>), grid, block, 0, st, pg, tab, env, K, dt, sa, beta, as, am, xb); break;
        case 4: hipLaunchKernelGGL((fused_plain_kernel<4, kFusedPPT, TRACK>), grid, block, 0, st, pg, tab, env, K, dt, sa, beta, as, am, xb); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fused_plain(const PointGeom& pg, int W, const SrcRec* tab, EnvSet env, int K, float dt, ScanArgs sa,
                              float* beta, float* as, float* am, double* xb, hipStream_t st) {
    if (pg.count <= 0) return hipSuccess;
    return xb ? fused_plain_w<true>(pg, W, tab, env, K, dt, sa, beta, as, am, xb, st)
              : fused_plain_w<false>(pg, W, tab, env, K, dt, sa, beta, as, am, xb, st);
}

// ---------------------------------------------------------------------------
// sample gather and invariant check
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void gather_kernel(const float* __restrict__ src, const int64_t* __restrict__ idx,
                                                       int64_t m, float* __restrict__ dst) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g < m) dst[g] = src[idx[g]];
}

hipError_t launch_gather(const float* src, const int64_t* idx, int64_t m, float* dst, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, src, idx, m,
                       dst);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void invariants_kernel(const float* __restrict__ beta, const float* __restrict__ as,
                                                           const float* __restrict__ am, const float* __restrict__ T,
                                                           int64_t n, float tol,
                                                           unsigned long long* __restrict__ counter) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool bad = false;
    if (g < n) {
        const float b = beta[g], a = as[g], m = am[g];
        bad = !(a >= -tol && a <= 1.0f + tol && m >= -tol && m <= 1.0f + tol && b >= -tol && b <= 1.0f + tol);
        bad = bad || !(a + m <= kXmax + tol);
        if (T) bad = bad || !(fabsf(a + m + b - solid_fraction(T[g])) <= tol);
    }
    // one atomic per wave
    const unsigned long long mask = __ballot(bad);
    if ((threadIdx.x & 63) == 0 && mask) atomicAdd(counter, (unsigned long long)__popcll(mask));
}

hipError_t launch_invariants(const float* beta, const float* as, const float* am, const float* T, int64_t n,
                             float tol, unsigned long long* counter, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(invariants_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, beta, as,
                       am, T, n, tol, counter);
    return hipGetLastError();
}

}  // namespace mstruct
