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
    int32_t k0;            // points on planes k < k0 are inactive
    float r2min;           // squared clamp radius around a switched-on source [grid units^2]
    float roff;            // radius around a switched-off track's virtual position [grid units]
};

// scan constants of one call
struct ScanArgs {
    float T0, Tclamp;
};

hipError_t launch_step(const float* Tp, const float* Tn, float* beta, float* as, float* am, int64_t n,
                       float dt, hipStream_t st);
hipError_t launch_fused_implicit(const PointGeom& pg, int W, const SrcRec* tab, int K, float h, int n_sub,
                                 int max_iter, ScanArgs sa, float* beta, float* as, float* am,
                                 unsigned long long* unconverged, hipStream_t st);
// float64 explicit step (step_f64_lib.hip: device math library; step_f64_synth.hip:
// exponent-bit exp2 / log2)
hipError_t launch_step_f64_library(const double* Tp, const double* Tn, double* beta, double* as, double* am,
                                   int64_t n, double dt, hipStream_t st);
hipError_t launch_step_f64_synth(const double* Tp, const double* Tn, double* beta, double* as, double* am,
                                 int64_t n, double dt, hipStream_t st);
hipError_t launch_implicit_step(const float* Tp, const float* Tn, float* beta, float* as, float* am, int64_t n,
                                float h, int n_sub, int max_iter, unsigned long long* unconverged,
                                hipStream_t st);
hipError_t launch_temperature(const PointGeom& pg, int W, const SrcRec* rec, ScanArgs sa, float* T,
                              hipStream_t st);
hipError_t launch_fused_plain(const PointGeom& pg, int W, const SrcRec* tab, int K, float dt, ScanArgs sa,
                              float* beta, float* as, float* am, hipStream_t st);
hipError_t launch_gather(const float* src, const int64_t* idx, int64_t m, float* dst, hipStream_t st);
hipError_t launch_invariants(const float* beta, const float* as, const float* am, const float* T, int64_t n,
                             float tol, unsigned long long* counter, hipStream_t st);

}  // namespace mstruct
