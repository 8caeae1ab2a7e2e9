// Learned surrogate (MLP 6 -> 64 -> 64 -> 3) state and launch interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace mstruct {

constexpr int kMlpIn = 6, kMlpHidden = 64, kMlpOut = 3;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpOut * kMlpHidden + kMlpOut;  // 4803

struct MlpState {
    bool ready = false;
};

void mlp_free(MlpState& s);
hipError_t launch_surrogate(const MlpState& s, const PointGeom& pg, int W, const SrcRec* tab, int K, float dt,
                            ScanArgs sa, float* beta, float* as, float* am, hipStream_t st);

}  // namespace mstruct
