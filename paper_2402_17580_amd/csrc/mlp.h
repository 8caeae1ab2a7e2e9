// Learned surrogate: MLP 6 -> 64 -> 64 -> 3 with ReLU, BF16 MFMA
// (v_mfma_f32_32x32x8_bf16) and float32 accumulation.  Not part of the paper:
// it replaces K explicit steps of a point by one network evaluation where an
// error indicator allows it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace mstruct {

constexpr int kMlpIn = 6, kMlpHidden = 64, kMlpOut = 3;
// flat float32 parameter vector: W1[64][6], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]
constexpr int kOffW1 = 0, kOffB1 = 384, kOffW2 = 448, kOffB2 = 4544, kOffW3 = 4608, kOffB3 = 4800;
constexpr int kMlpParams = 4803;

// per-lane MFMA operand fragments, stored word-major (word w of lane l at w * 64 + l)
constexpr int kFragW1 = 0;     // [mt 2][2 words]
constexpr int kFragW2 = 4;     // [mt 2][kb 8][2 words]
constexpr int kFragW3 = 36;    // [kb 8][2 words]
constexpr int kFragW3T = 52;   // [mt 2][2 words]     (backward)
constexpr int kFragW2T = 56;   // [mt 2][kb 8][2 words] (backward)
constexpr int kFragB2 = 88;    // [mt 2][16] float accumulator init
constexpr int kFragB3 = 120;   // [16] float accumulator init
// inference operands for v_mfma_f32_32x32x16_bf16 (K index permuted, see mlp.hip)
constexpr int kFragI2 = 136;   // [mt 2][kb 4][4 words]
constexpr int kFragI3 = 168;   // [kb 4][4 words]
constexpr int kFragWords = 184;
constexpr int kFragUniform = kFragWords * 64;  // then b3[3] as plain floats
constexpr int kFragTotal = kFragUniform + 16;

// normalisation and error-indicator constants (host-set)
struct MlpNorm {
    float in_mean[kMlpIn];
    float in_inv_scale[kMlpIn];
    float out_scale[kMlpOut];
    float T_cold;    // blocks entirely below this temperature may use the network
    float T_hot_lo;  // ... or entirely inside [T_hot_lo, T_hot_hi]
    float T_hot_hi;
    float dT_max;    // |T_end - T_start| above this forces the plain steps
};

struct MlpState {
    bool ready = false;
    MlpNorm norm{};
    float* master = nullptr;   // float32 parameters
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    float* grad = nullptr;     // reduced gradient
    float* loss = nullptr;     // reduced loss
    uint32_t* frag = nullptr;  // bf16 fragments (+ float bias words), kFragTotal words
    float* partial = nullptr;  // per-wave partial gradients [waves][kMlpParams + 1]
    int partial_waves = 0;
    int adam_t = 0;
    // surrogate mode: records of the waves that stop for the network (see
    // mlp.hip), and two record counters used by alternate launches
    void* recs = nullptr;
    int64_t rec_cap = 0;
    unsigned* counters = nullptr;
};

hipError_t mlp_alloc(MlpState& s);
void mlp_free(MlpState& s);
hipError_t mlp_pack(const MlpState& s, hipStream_t st);
hipError_t mlp_forward(const MlpState& s, const float* X, int64_t B, float* Y, hipStream_t st);
hipError_t mlp_grad(MlpState& s, const float* X, const float* Y, int64_t B, float* grad, float* loss,
                    hipStream_t st);
hipError_t mlp_adam(MlpState& s, float lr, hipStream_t st);
// before the launches of a surrogate call on `waves` waves of 64 points
hipError_t surrogate_prepare(MlpState& s, int64_t waves, hipStream_t st);
// one launch of Kl steps (launch li of the call) in blocks of Ks steps, with
// the launch certificates and wave flags of env as in the plain fused launch
// SURROGATE launches l0 .. l0 + nl - 1 of a call with wave flags: the list
// pass, fused_surrogate_call_kernel (no network; waves that need it are
// recorded) and surrogate_resume_call_kernel (the recorded waves to the end of
// the chunk, with the network); arguments as for launch_fused_plain_call, Kl
// steps per launch, networks of Ks steps
hipError_t launch_surrogate_call(const MlpState& s, const PointGeom& pg, int W, const SrcRec* tab, const EnvRec* env,
                                 const int32_t* env_fc, const uint8_t* below, uint8_t* rest, int64_t n_waves,
                                 int64_t l0, int64_t nl, int Kl, int Ks, int64_t n_steps, float dt, ScanArgs sa,
                                 float* beta, float* as, float* am, uint32_t* cand, unsigned* counts,
                                 unsigned long long* stats, hipStream_t st);
hipError_t launch_surrogate(const MlpState& s, const PointGeom& pg, int W, const SrcRec* tab, EnvSet env, int Kl,
                            int Ks, float dt, ScanArgs sa, float* beta, float* as, float* am, int64_t li,
                            hipStream_t st);
hipError_t launch_correct(const float* T, float* beta, float* as, float* am, int64_t n, bool assign, hipStream_t st);

}  // namespace mstruct
