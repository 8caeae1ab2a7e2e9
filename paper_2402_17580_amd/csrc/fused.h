// Shared pieces of the fused kernels (plain, implicit and surrogate): point
// decoding, the launch certificates' wave tests, the persistent slot form of
// a launch, the per-wave flags and counts.
#pragma once
#include "kernels.h"

namespace mstruct {

// workgroup of the fused grid kernels (one wave per 64 points)
constexpr int kFusedBlock = 256;
// wave slots per wave of the persistent fused kernels (see fused_slots),
// and the launch size (in waves) from which they run in workgroups of four
// waves instead of two: on large, mostly still grids the occupancy of four
// pays (island block, 1M waves: 2.2 s against 2.7 s), on smaller ones two
// spread the waves that step over more CUs (block scan, 131k waves: 9 %
// faster)
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

// The list form of a slot launch: the waves of the launch that are not
// still by their flags, listed by candidates_kernel (which also wrote beta
// for the still ones); wave p of the grid takes the entries p, p + P, ...
// (P waves in the grid).  Consecutive entries, which are neighbouring waves
// of points, go to consecutive waves of the grid and so to different CUs,
// and every wave that steps is launched at the start of the kernel.
template <int BS, class Body>
__device__ __forceinline__ void fused_list(const EnvSet& env, Body body) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *env.cand_next = 0u;
    const int64_t n = *env.cand_n;
    const int64_t P = (int64_t)gridDim.x * (BS / kWave);
    const int64_t p = (int64_t)blockIdx.x * (BS / kWave) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    for (int64_t e = p; e < n; e += P) body((int64_t)__builtin_amdgcn_readfirstlane((int)env.cand[e]));
}

// The persistent form of a fused launch, used from the second launch of a
// call when the wave flags are kept: a grid of about one wave per
// slots_per_wave waves of the launch, in which wave p takes the wave slots p,
// p + P, p + 2P, ... (P waves in the grid).  Each lane loads the flags of
// one slot; the wave then runs body(w) for every slot w that is not still
// (all 64 lanes, one point each) and writes beta for the still ones.  No
// wave is launched only to find its flags set, and the interleaved slots
// spread the few waves that step evenly over the grid.  With a list of the
// waves that step (EnvSet::cand), the launch takes its list form instead.
template <int BS, class Body>
__device__ __forceinline__ void fused_slots(const PointGeom& pg, const EnvSet& env, float T0c, float* beta,
                                            Body body) {
    if (env.cand) {  // the launch's list of the waves that step
        fused_list<BS>(env, body);
        return;
    }
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t P = (int64_t)gridDim.x * (BS / kWave);
    const int64_t p = (int64_t)blockIdx.x * (BS / kWave) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    for (int64_t r = 0; p + r * kWave * P < env.n_waves; ++r) {
        const int64_t w = p + (r * kWave + lane) * P;
        const bool in = w < env.n_waves;
        const bool still = in && env.below[w] && env.rest[w];
        uint64_t todo = __ballot(in && !still), quiet = beta ? __ballot(still) : 0;
        if (env.stats) {
            const int nq = __popcll(__ballot(still));  // (all lanes take part in the ballot)
            if (nq && lane == 0) atomicAdd(env.stats + kStatFlagged, (unsigned long long)nq);
        }
        while (todo) {
            const int i = __builtin_ctzll(todo);
            todo &= todo - 1;
            body(p + (r * kWave + i) * P);
        }
        while (quiet) {
            const int i = __builtin_ctzll(quiet);
            quiet &= quiet - 1;
            still_wave_beta(pg, T0c, beta, (p + (r * kWave + i) * P) * kWave + lane);
        }
    }
}

// count a wave that read its state: its active points, and its class
__device__ __forceinline__ void count_wave(const EnvSet& env, bool act, bool still, bool cold) {
    const unsigned long long n = __popcll(__ballot(act));
    if ((threadIdx.x & (kWave - 1)) != 0 || n == 0) return;
    atomicAdd(env.stats + kStatLoaded, n);
    if (still) {
        atomicAdd(env.stats + kStatStill, 1ull);
        return;
    }
    atomicAdd(env.stats + kStatStored, n);
    atomicAdd(env.stats + (cold ? kStatCold : kStatHot), 1ull);
}

// count a hot wave's sub-block from T0 to TK, and whether every point passes
// the surrogate's default indicator on it
__device__ __forceinline__ void count_block(const EnvSet& env, bool act, float T0, float TK) {
    const float lo = fminf(T0, TK), hi = fmaxf(T0, TK);
    const bool ok = !act || ((hi < 823.0f || (lo >= 1398.0f && hi <= 1853.0f)) && fabsf(TK - T0) <= 50.0f);
    const bool all = __ballot(!ok) == 0;
    if ((threadIdx.x & (kWave - 1)) != 0) return;
    atomicAdd(env.stats + kStatHotBlocks, 1ull);
    if (all) atomicAdd(env.stats + kStatEligibleBlocks, 1ull);
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

// Wave slots per wave of a slot kernel.  Below kSlotsLargeGrid waves, four
// (sixteen took the block scan from 62 to 101 ms).  On large grids, where
// nearly every wave exits on its flags, fewer slot waves cut the cost of
// launching them when the waves that step run short chains: 16 for plain
// launches of at most 16 steps (masked cantilever, K = 16: 0.32 -> 0.19 s
// per run), 8 for the surrogate, whose admitted blocks take one step (island
// block: 0.643 -> 0.607 s); plain launches of more steps keep four (island
// block at K = 64: 1.84 s, 2.01 s with 16).
enum class SlotUse { PlainShort, PlainLong, Surrogate, Implicit };
inline int slots_per_wave(int64_t n_waves, SlotUse use) {
    if (n_waves < kSlotsLargeGrid) return kSlotsPerWave;
    return use == SlotUse::PlainShort ? 16 : use == SlotUse::Surrogate ? 8 : kSlotsPerWave;
}

}  // namespace mstruct
