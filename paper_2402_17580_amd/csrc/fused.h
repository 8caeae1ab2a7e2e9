// Shared pieces of the fused kernels (plain, implicit and surrogate): point
// decoding, the launch certificates' wave tests, the persistent slot form of
// a launch, the per-wave flags and counts.
#pragma once
#include "kernels.h"

namespace mstruct {

// workgroup of the fused grid kernels (one wave per 64 points)
constexpr int kFusedBlock = 256;
// waves of points per grid wave of the slot kernels (see fused_slots and
// slots_per_wave), and the launch size (in waves of points) from which their
// workgroups hold four waves instead of two
constexpr int kSlotsPerWave = 4;
constexpr int64_t kSlotsLargeGrid = (int64_t)1 << 18;

// grid coordinates of a local point number (box or index list)
__device__ __forceinline__ void decode_point(const PointGeom& pg, int64_t local, int& gi, int& gj, int& gk) {
    const int lin = pg.index ? pg.index[local] : (int)local;
    gk = divide_by(lin, pg.mag_nxy, pg.sh_nxy);
    const int rem = lin - gk * pg.nxy;
    gj = divide_by(rem, pg.mag_nx, pg.sh_nx);
    gi = rem - gj * pg.nx;
}

// The point at position g (0 <= g < count) of a call's wave order (wave w:
// positions 64 w .. 64 w + 63): its array index, and its grid coordinates.
// On an index list, and on a box grid without tiles, the order is that of
// the arrays.  On a tiled box grid (tiles of a = 2^tw_log by b = 64 / a
// points), position q = first + g lies on plane q / (nx ny), and the
// positions of a plane run through its tiles row by row, 64 per tile, lane
// l of a tile at (a tx + l % a, b ty + l / a): the waves along a track then
// cover fewer points that need not step than parts of rows would when the
// track does not run along x.
__device__ __forceinline__ int64_t point_at(const PointGeom& pg, int64_t g, int& gi, int& gj, int& gk) {
    const int64_t q = pg.first + g;
    if (!pg.tiled) {
        decode_point(pg, q, gi, gj, gk);
        return q;
    }
    const int lin = (int)q;
    gk = divide_by(lin, pg.mag_nxy, pg.sh_nxy);
    const int r = lin - gk * pg.nxy, t = r >> 6, l = r & 63;
    const int ty = divide_by(t, pg.mag_tr, pg.sh_tr);
    gi = ((t - ty * pg.tr) << pg.tw_log) + (l & ((1 << pg.tw_log) - 1));
    gj = (ty << (6 - pg.tw_log)) + (l >> pg.tw_log);
    return (int64_t)gk * pg.nxy + (int64_t)gj * pg.nx + gi;
}

// squared distance [grid units^2] within which the envelope tests certify
// nothing: one grid unit, and at least the clamp radius and the offset
// radius of source_rise
__host__ __device__ __forceinline__ float envelope_radius2(const PointGeom& pg) {
    return fmaxf(1.0f, fmaxf(pg.roff * pg.roff, pg.r2min));
}

// limit of the still test: the alpha_s -> beta end temperature of at_rest,
// with 0.5 K to spare for float32 rounding of the computed temperatures
constexpr float kRestBelow = Const<float>::TasEnd - 0.5f;

// whether the still test can succeed (wave-uniform): certificates enabled,
// T0 below the limit and every point of the wave at rest at the start of
// the launch
__device__ __forceinline__ bool wave_may_rest(const EnvSet& env, bool act, float a, float m, float T0) {
    return env.n >= 0 && T0 < kRestBelow && __ballot(act && !rest_bits(a, m)) == 0;
}

// whether the box pre-pass (still_flags_kernel) bounded wave wv below the
// still limit at every time point of this launch: then a wave whose points
// are all at rest is still without the per-point bounds of wave_below
__device__ __forceinline__ bool wave_box_below(const EnvSet& env, int64_t wv) {
    return env.below && wv < env.n_waves && env.below[wv];
}

// A cold wave (T = T0 at every step) whose first explicit step of a launch
// left a point's fractions x0 (alpha_s, alpha_m) with the same bits, with lo
// the compensated low part after that step (its increment, or 0 where the
// correction reset it).  Every later step then starts from the same high
// parts at the same temperature, takes the same increments and gives the
// correction the same input: a low part that stays below a quarter of the
// float spacing around x0 keeps x0 + lo rounding to x0 at every step and at
// the end.  K |lo| <= 2^(e - 27) for x0 = f 2^e, f in [0.5, 1), is half of
// that (covering the rounding of the K additions); x0 = 0 needs lo = 0 and
// x0 = +0.0, so that the final x0 + lo has the bits of x0.  Then the K steps
// leave the stored fractions as they are, bit for bit (frozen): at the
// 300 K of material far from the tracks the rates are of order 1e-9 / s.
__device__ __forceinline__ bool frozen_part(float x0, float x1, float lo, int K) {
    if (__float_as_uint(x1) != __float_as_uint(x0)) return false;
    if (x0 == 0.0f) return lo == 0.0f && __float_as_uint(x0) == 0u;
    return lo == 0.0f || (float)K * fabsf(lo) <= ldexpf(1.0f, __builtin_amdgcn_frexp_expf(x0) - 27);
}

// wave index of the calling lane in a fused launch (uniform across the wave)
__device__ __forceinline__ int64_t fused_wave() {
    return (int64_t)blockIdx.x * (kFusedBlock / kWave) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

// A wave whose flags say still (wave_flag_still): its state is at rest and
// stays as it is, so only beta (last launch of a call) is written, with the
// value every step would give.
// On an index list, points above the current surface are inactive and left
// alone (on a box grid every point of a call is active).
__device__ __forceinline__ void still_wave_beta(const PointGeom& pg, float T0c, float* beta, int64_t g) {
    if (!beta || g >= pg.count) return;
    int gi, gj, gk;
    const int64_t local = point_at(pg, g, gi, gj, gk);
    if (pg.index && gk < pg.k0) return;
    beta[local] = solid_fraction(T0c) - kXmax - 0.0f;
}

// A slot launch: the waves of the launch that are not still by their flags,
// listed by candidates_kernel or first_candidates_kernel (which also wrote
// beta for the still ones) in env.cand[0 .. *env.cand_n), taken by a grid of
// about one wave per slots_per_wave waves of points: wave p of the grid takes
// the entries p, p + P, ... (P waves in the grid) and runs body(w) for each
// (all 64 lanes, one point each).  Consecutive entries, which are
// neighbouring waves of points, go to consecutive waves of the grid and so to
// different CUs, and every wave that steps starts with the kernel.  The
// launch clears *env.cand_next, the next launch's count.
template <int BS, class Body>
__device__ __forceinline__ void fused_slots(const EnvSet& env, Body body) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *env.cand_next = 0u;
    const int64_t n = *env.cand_n;
    const int64_t P = (int64_t)gridDim.x * (BS / kWave);
    const int64_t p = (int64_t)blockIdx.x * (BS / kWave) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    for (int64_t e = p; e < n; e += P) body((int64_t)__builtin_amdgcn_readfirstlane((int)env.cand[e]));
}

// The counts below are added by every lane, lane 0 with the value and the
// others with 0, so that no branch on the lane sits inside the kernels'
// loops (see fused_plain_call_kernel).

// count a wave that read its state: its active points, and its class
__device__ __forceinline__ void count_wave(const EnvSet& env, bool act, bool still, bool cold) {
    const unsigned long long n = __popcll(__ballot(act));
    if (n == 0) return;  // (uniform)
    const unsigned long long one = (threadIdx.x & (kWave - 1)) == 0 ? 1ull : 0ull;
    atomicAdd(env.stats + kStatLoaded, n * one);
    if (still) {
        atomicAdd(env.stats + kStatStill, one);
        return;
    }
    atomicAdd(env.stats + kStatStored, n * one);
    atomicAdd(env.stats + (cold ? kStatCold : kStatHot), one);
}

// count a hot wave's sub-block from T0 to TK, and whether every point passes
// the surrogate's default indicator on it
__device__ __forceinline__ void count_block(const EnvSet& env, bool act, float T0, float TK) {
    const float lo = fminf(T0, TK), hi = fmaxf(T0, TK);
    const bool ok = !act || ((hi < 823.0f || (lo >= 1398.0f && hi <= 1853.0f)) && fabsf(TK - T0) <= 50.0f);
    const bool all = __ballot(!ok) == 0;
    const unsigned long long one = (threadIdx.x & (kWave - 1)) == 0 ? 1ull : 0ull;
    atomicAdd(env.stats + kStatHotBlocks, one);
    if (all) atomicAdd(env.stats + kStatEligibleBlocks, one);
}

// record whether every point of the wave is at rest after the launch
__device__ __forceinline__ void record_rest(const EnvSet& env, int64_t wv, bool act, float a, float m) {
    if (!env.below || wv >= env.n_waves) return;
    const bool r = __ballot(act && !rest_bits(a, m)) == 0;
    if ((threadIdx.x & (kWave - 1)) == 0) env.rest[wv] = r ? 1 : 0;
}

// grid of the persistent (slot) fused kernels in workgroups of bs threads:
// one wave per spw waves of the launch
inline dim3 slots_grid(int64_t n_waves, int bs, int spw) {
    const int64_t waves = (n_waves + spw - 1) / spw;
    return dim3((unsigned)((waves + bs / kWave - 1) / (bs / kWave)));
}

// launch a slot kernel instantiated for workgroups of 128 and 256 threads,
// spw wave slots per wave
#define LAUNCH_SLOTS(kernel, W, n_waves, spw, st, ...)                                                          \
    do {                                                                                                         \
        if ((n_waves) >= kSlotsLargeGrid)                                                                        \
            hipLaunchKernelGGL((kernel<W, 256>), slots_grid(n_waves, 256, spw), dim3(256), 0, st, __VA_ARGS__); \
        else                                                                                                     \
            hipLaunchKernelGGL((kernel<W, 128>), slots_grid(n_waves, 128, spw), dim3(128), 0, st, __VA_ARGS__); \
    } while (0)

// Waves of points per grid wave of a slot kernel (IMPLICIT launches): the
// grid only has to hold the listed waves, a few per cent of a launch (from
// 4 to 32 within 1 %; 2 was 6-9 % slower on the large grids).
inline int slots_per_wave(int64_t) { return kSlotsPerWave; }

}  // namespace mstruct
