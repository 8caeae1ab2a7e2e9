// Kernel launch interface shared by the C-ABI layer and the kernel sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "heat_source.h"

namespace mstruct {

// the active points of one call
struct PointGeom {
    const int32_t* index;  // box linear indices, or nullptr for the whole box
    int64_t first;         // first local point number processed
    int64_t count;         // number of local points processed
    int32_t nx, nxy;       // box dimensions
    // exact division by nx and nxy for 0 <= n < 2^31: n / d = mulhi(n, mag) >> sh
    // (sh < 0 marks d = 1); see divide_magic
    uint32_t mag_nx, mag_nxy;
    int32_t sh_nx, sh_nxy;
    int32_t k0;            // points on planes k < k0 are inactive
    // tiled != 0 (box grid only): the waves of the fused kernels take tiles of
    // 2^tw_log x 2^(6 - tw_log) points of a plane (see point_at); tr tiles
    // per row, divided by with (mag_tr, sh_tr)
    int32_t tiled, tw_log, tr;
    uint32_t mag_tr;
    int32_t sh_tr;
    float r2min;           // squared clamp radius around a switched-on source [grid units^2]
    float roff;            // radius around a switched-off track's virtual position [grid units]
};

// floor(n / d) for 0 <= n < 2^31 from the multiplier and shift of divide_magic
__device__ __forceinline__ int32_t divide_by(int32_t n, uint32_t mag, int32_t sh) {
    return sh < 0 ? n : (int32_t)(__umulhi((uint32_t)n, mag) >> sh);
}

// Multiplier and shift for exact unsigned division of n < 2^31 by d >= 1:
// with l = ceil(log2 d) >= 1, mag = ceil(2^(31+l) / d) < 2^32 and
// n / d = (n mag) >> (31 + l); the error n (mag - 2^(31+l)/d) / 2^(31+l) is
// below 2^-l <= 1/d, so the floor is exact.  d = 1 gives sh = -1.
inline void divide_magic(int64_t d, uint32_t& mag, int32_t& sh) {
    if (d <= 1) {
        mag = 0;
        sh = -1;
        return;
    }
    int l = 0;
    while (((int64_t)1 << l) < d) ++l;
    mag = (uint32_t)((((uint64_t)1 << (31 + l)) + (uint64_t)d - 1) / (uint64_t)d);
    sh = l - 1;
}

// scan constants of one call, and the context's readings of the paper
struct ScanArgs {
    float T0, Tclamp;
    Readings rd;
};

// the envelope records of one launch (see EnvRec), and the per-wave flags of
// a box grid (below == nullptr: not used; never with a tracked X~beta):
// below[w] != 0 when still_flags bounded every point of wave w below the
// still limit through this launch; rest[w] != 0 when every point of wave w
// was at rest after the last launch that took its steps.  rest is read only
// when read_rest (from the second launch of a call) and written by every
// wave that takes its steps.
struct EnvSet {
    const EnvRec* rec;
    int32_t n;
    const uint8_t* below;
    uint8_t* rest;
    int64_t n_waves;
    int32_t read_rest;
    // wave counts of fused PLAIN / IMPLICIT launches (nullptr: not counted),
    // indexed by the kStat* constants
    unsigned long long* stats;
    // the waves of a slot launch that are not still by their flags, listed
    // by candidates_kernel (cand[0 .. *cand_n)); the slot kernels run only
    // with a list (nullptr: the grid kernels, which read the flags
    // themselves).  The slot launch clears *cand_next, the next launch's
    // count.
    uint32_t* cand;
    unsigned* cand_n;
    unsigned* cand_next;
};

// the counts of EnvSet::stats: points whose state a launch reads and writes,
// and its waves by class (still by the certificates after reading the state,
// cold, hot: the temperature evaluated at every step, still by the wave
// flags without reading the state); then, for fused PLAIN launches, the hot
// waves' whole sub-blocks of kStatBlock steps, and those of them in which
// every point passes the surrogate's default error indicator (both
// sub-block-end temperatures below 823 K or both within [1398, 1853] K, at
// most 50 K apart): the share of hot-wave steps the network may replace
enum { kStatLoaded = 0, kStatStored = 1, kStatStill = 2, kStatCold = 3, kStatHot = 4, kStatFlagged = 5,
       kStatHotBlocks = 6, kStatEligibleBlocks = 7, kStatCount = 8 };
constexpr int kStatBlock = 8;

// points per wave of the fused kernels (one point per lane)
constexpr int kWave = 64;

// a state at rest with alpha_m = +0.0 exactly: steps at rest store m + 0 =
// +0.0, so a wave of such states may skip its stores
__device__ __forceinline__ bool rest_bits(float a, float m) { return a == kXmax && __float_as_uint(m) == 0u; }

// wave wv (points 64 wv .. 64 wv + 63) is still by its flags: bounded below
// the still limit through this launch and at rest after the previous one
__device__ __forceinline__ bool wave_flag_still(const EnvSet& env, int64_t wv) {
    return env.below && env.read_rest && wv < env.n_waves && env.below[wv] && env.rest[wv];
}

// still_flags for launches l0 .. l0 + nl - 1 of a call on a box grid:
// flags[(l - l0) * n_waves + w] for wave w = points 64 w .. 64 w + 63 of pg;
// env_fc holds (first record, count) of each launch's envelopes in env.
// boxes: the box of each wave followed by the box of each group of 64 waves
// (launch_wave_boxes), or nullptr on a box grid without an index list, where
// they follow from the first and last points.
hipError_t launch_still_flags(const PointGeom& pg, const EnvRec* env, const int32_t* env_fc, int64_t l0, int64_t nl,
                              int64_t n_waves, float T0, const GridBox* boxes, uint8_t* flags, hipStream_t st);

// groups of 64 waves (4096 points) whose common box the still-flag pre-pass
// tests first
__host__ __device__ inline int64_t wave_groups(int64_t n_waves) { return (n_waves + 63) / 64; }

// boxes[w]: the box of grid positions of the points 64 w .. 64 w + 63 of pg
// (any index list: the least and greatest coordinates of its points), then
// boxes[n_waves + s]: the box of waves 64 s .. 64 s + 63 (n_waves +
// wave_groups(n_waves) boxes in all)
hipError_t launch_wave_boxes(const PointGeom& pg, int64_t n_waves, GridBox* boxes, hipStream_t st);

// list the waves of a slot launch that are not still by their flags into
// env.cand (count in *env.cand_n), and write beta (if not nullptr) for the
// still ones; clear_counts zeroes the two counts of a call
hipError_t launch_candidates(const PointGeom& pg, const EnvSet& env, float T0c, float* beta, hipStream_t st);
// the same for the first launch of a call, from the state (as, am) and the
// box pre-pass's flags; sets the rest flags of the still waves
hipError_t launch_first_candidates(const PointGeom& pg, const EnvSet& env, float T0c, float* beta, const float* as,
                                   const float* am, hipStream_t st);
hipError_t launch_clear_counts(unsigned* counts, hipStream_t st);

// xb: optional tracked X~beta side values (float64 per point), or nullptr
hipError_t launch_step(const float* Tp, const float* Tn, float* beta, float* as, float* am, double* xb, int64_t n,
                       float dt, Readings rd, hipStream_t st);
hipError_t launch_fused_implicit(const PointGeom& pg, int W, const SrcRec* tab, EnvSet env, int K, float h, int n_sub,
                                 int max_iter, ScanArgs sa, float* beta, float* as, float* am, double* xb,
                                 unsigned long long* unconverged, hipStream_t st);
// float64 explicit step (step_f64_lib.hip: device math library; step_f64_synth.hip:
// exponent-bit exp2 / log2)
// (the readings as plain flags: these translation units have their own model namespaces)
hipError_t launch_step_f64_library(const double* Tp, const double* Tn, double* beta, double* as, double* am,
                                   int64_t n, double dt, bool corr_prev, bool mart_assign, hipStream_t st);
hipError_t launch_step_f64_synth(const double* Tp, const double* Tn, double* beta, double* as, double* am,
                                 int64_t n, double dt, bool corr_prev, bool mart_assign, hipStream_t st);
// step_f64_paper.hip: the paper's exp / ln (bit synthesis with its correction polynomials)
hipError_t launch_step_f64_paper(const double* Tp, const double* Tn, double* beta, double* as, double* am,
                                 int64_t n, double dt, bool corr_prev, bool mart_assign, hipStream_t st);
// the implicit scheme corrects at T^{n+1}: only rd.mart_assign applies
hipError_t launch_implicit_step(const float* Tp, const float* Tn, float* beta, float* as, float* am, double* xb,
                                int64_t n, float h, int n_sub, int max_iter, unsigned long long* unconverged,
                                Readings rd, hipStream_t st);
hipError_t launch_temperature(const PointGeom& pg, int W, const SrcRec* rec, ScanArgs sa, float* T,
                              hipStream_t st);
hipError_t launch_fused_plain(const PointGeom& pg, int W, const SrcRec* tab, EnvSet env, int K, float dt, ScanArgs sa,
                              float* beta, float* as, float* am, double* xb, hipStream_t st);
// fused PLAIN launches l0 .. l0 + nl - 1 of a call with wave flags: a list
// pass (chunk_list_kernel) and one persistent kernel (fused_plain_call_kernel)
// for the listed waves.  tab and env_fc as for the whole call, below the
// chunk's still flags, rest one byte per wave, cand room for n_waves
// entries, counts two counters (cleared here); beta (nullptr: not written)
// when the chunk ends the call
hipError_t launch_fused_plain_call(const PointGeom& pg, int W, const SrcRec* tab, const EnvRec* env,
                                   const int32_t* env_fc, const uint8_t* below, uint8_t* rest, int64_t n_waves,
                                   int64_t l0, int64_t nl, int K, int64_t n_steps, float dt, ScanArgs sa, float* beta,
                                   float* as, float* am, uint32_t* cand, unsigned* counts,
                                   unsigned long long* stats, hipStream_t st);
// the list pass of a chunk of launches l0 .. l0 + nl - 1 (chunk_list_kernel):
// the waves that are not still throughout the chunk in cand[0 .. counts[0]);
// counts[0] and counts[1] cleared first
hipError_t launch_chunk_list(const PointGeom& pg, const uint8_t* below, uint8_t* rest, int64_t n_waves, int64_t l0,
                             int64_t nl, float T0c, float* beta, const float* as, const float* am, uint32_t* cand,
                             unsigned* counts, unsigned long long* stats, hipStream_t st);
// workgroup and grid of the persistent call kernels (kCallBlock threads,
// kCallWaves grid waves at most: eight per SIMD)
constexpr int kCallBlock = 256;
dim3 call_grid(int64_t n_waves);
hipError_t launch_gather(const float* src, const int64_t* idx, int64_t m, float* dst, hipStream_t st);
hipError_t launch_invariants(const float* beta, const float* as, const float* am, const float* T, int64_t n,
                             float tol, unsigned long long* counter, hipStream_t st);

}  // namespace mstruct
