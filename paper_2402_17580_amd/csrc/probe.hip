// Calibration probes for the VALU roofline (a library of its own,
// libmstruct_probe.so; not part of the phase-update library).
//
// Each lane runs `iters` iterations of 8 independent dependency chains of one
// VALU instruction each, so a wave issues exactly 8 iters (kind 0 or 1) or
// 16 iters (kind 2) VALU instructions in its loop (loop control is scalar):
//   kind 0  v_fma_f32   x = x * 0.999 + 0.001       (full-rate VOP3)
//   kind 1  v_exp_f32   x = 2^-x                    (transcendental)
//   kind 2  both, interleaved, on 16 independent chains
// Timing a launch gives wave64 instructions per second; rocprofv3 counters of
// the same launch give what SQ_INSTS_VALU and the busy-cycle counters report
// for a known instruction count.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mstruct_probe {

constexpr int kThreads = 256;

template <int KIND>
__global__ __launch_bounds__(kThreads) void valu_probe_kernel(int iters, float* __restrict__ out) {
    const int g = blockIdx.x * kThreads + threadIdx.x;
    float x[8], y[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        x[c] = 0.5f + 0.01f * (float)((g + c) & 31);
        y[c] = 0.25f + 0.01f * (float)((g + 3 * c) & 31);
    }
#pragma unroll 1
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (KIND == 0 || KIND == 2) x[c] = fmaf(x[c], 0.999f, 0.001f);
            if (KIND == 1) x[c] = __builtin_amdgcn_exp2f(-x[c]);
            if (KIND == 2) y[c] = __builtin_amdgcn_exp2f(-y[c]);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += x[c] + y[c];
    out[g] = s;
}

}  // namespace mstruct_probe

using namespace mstruct_probe;

extern "C" {

// Launch `blocks` workgroups of 256 threads of probe `kind` (0, 1, 2) with
// `iters` loop iterations; out: device float32 [blocks * 256].  Returns 0,
// or -1 for a bad argument, -2 for a launch error.
int probe_valu(int kind, int iters, int blocks, float* out, void* stream) {
    if (kind < 0 || kind > 2 || iters < 1 || blocks < 1 || !out) return -1;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)blocks), block(kThreads);
    switch (kind) {
        case 0: hipLaunchKernelGGL(valu_probe_kernel<0>, grid, block, 0, st, iters, out); break;
        case 1: hipLaunchKernelGGL(valu_probe_kernel<1>, grid, block, 0, st, iters, out); break;
        default: hipLaunchKernelGGL(valu_probe_kernel<2>, grid, block, 0, st, iters, out); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// VALU instructions one wave issues in the loop of probe `kind`
int64_t probe_valu_insts_per_wave(int kind, int iters) { return (int64_t)(kind == 2 ? 16 : 8) * iters; }

}  // extern "C"
