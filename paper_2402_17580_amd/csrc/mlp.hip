// Surrogate MLP kernels for gfx950: inference fused into the K-step update,
// and training (forward + backward + deterministic gradient reduction + Adam).
//
// All products use v_mfma_f32_32x32x8_bf16 (A 32x8, B 8x32, C 32x32).  With
// h = lane / 32 and j = lane % 32, lane l supplies A[j][4h..4h+3] and
// B[4h..4h+3][j] and holds C[(r%4) + 4h + 8(r/4)][j] in accumulator r.  A layer
// is computed transposed, features x points: its accumulator rows 8kb..8kb+7
// of column j sit in registers 4kb..4kb+3 of lanes j and j+32 in exactly the
// order the next layer's B operand for k-block kb needs, so activations pass
// from layer to layer in registers (after ReLU and conversion to bf16).
//
// Inference uses v_mfma_f32_32x32x16_bf16 for the two 64-wide layers (lane l
// supplies B[8h..8h+7][j]).  A C tile's registers 8q..8q+7 of lane half h hold
// features 16q + 4h + {0..3} and 16q + 8 + 4h + {0..3}; the product sums over
// k, so the same permutation of k is applied to the weights and those eight
// registers become the B operand as they are.
#include "fused.h"
#include "mlp.h"


namespace mstruct {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef short s2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    const bf2v v = __builtin_convertvector((f2v){a, b}, bf2v);  // round to nearest even
    return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ s4 make_s4(uint32_t lo, uint32_t hi) { return __builtin_bit_cast(s4, (u2v){lo, hi}); }
__device__ __forceinline__ f16v mfma(s4 a, s4 b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ float bf16_bits_to_float(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ f16v mfma16(bf8v a, bf8v b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// ReLU of two packed bf16 values: as 16-bit integers every negative value
// (and -0) is below 0, so an integer max with 0 zeroes exactly those
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t w) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s2v, w), (s2v){0, 0}));
}
// feature carried by item i of lane half h in the 16-wide k-block kb of a
// chained operand (the order in which an accumulator tile holds its rows)
__host__ __device__ __forceinline__ int chained_feature(int kb, int h, int i) {
    return 16 * kb + 4 * h + (i & 3) + ((i >> 2) << 3);
}

struct FwdFrag {
    s4 w1[2];
    s4 w2[2][8];
    s4 w3[8];
    f16v b2[2];
    f16v b3;
};

__device__ __forceinline__ s4 frag_s4(const uint32_t* __restrict__ frag, int word, int lane) {
    return make_s4(frag[word * 64 + lane], frag[(word + 1) * 64 + lane]);
}

__device__ __forceinline__ void load_fwd_frag(FwdFrag& F, const uint32_t* __restrict__ frag, int lane) {
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        F.w1[mt] = frag_s4(frag, kFragW1 + 2 * mt, lane);
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) F.w2[mt][kb] = frag_s4(frag, kFragW2 + 2 * (mt * 8 + kb), lane);
#pragma unroll
        for (int r = 0; r < 16; ++r) F.b2[mt][r] = __uint_as_float(frag[(kFragB2 + mt * 16 + r) * 64 + lane]);
    }
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) F.w3[kb] = frag_s4(frag, kFragW3 + 2 * kb, lane);
#pragma unroll
    for (int r = 0; r < 16; ++r) F.b3[r] = __uint_as_float(frag[(kFragB3 + r) * 64 + lane]);
}

// ReLU of accumulator registers r0..r0+3 packed as a bf16 B operand
__device__ __forceinline__ s4 relu_pack(const f16v& d, int r0) {
    return make_s4(pack_bf16x2(fmaxf(d[r0], 0.0f), fmaxf(d[r0 + 1], 0.0f)),
                   pack_bf16x2(fmaxf(d[r0 + 2], 0.0f), fmaxf(d[r0 + 3], 0.0f)));
}

// forward of one tile of 32 points: xb = input B operand (inputs 4h..4h+3 of
// point j); returns layer-3 accumulators (outputs in rows 0..2 = registers
// 0..2 of lanes with h = 0); h1, h2 receive the bf16 activations
__device__ __forceinline__ f16v forward_tile(const FwdFrag& F, s4 xb, s4 h1[8], s4 h2[8]) {
    const f16v zero = {};
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const f16v d = mfma(F.w1[mt], xb, zero);
#pragma unroll
        for (int q = 0; q < 4; ++q) h1[mt * 4 + q] = relu_pack(d, 4 * q);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f16v acc = F.b2[mt];
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) acc = mfma(F.w2[mt][kb], h1[kb], acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) h2[mt * 4 + q] = relu_pack(acc, 4 * q);
    }
    f16v o = F.b3;
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) o = mfma(F.w3[kb], h2[kb], o);
    return o;
}

// network on the 64 points of a wave, one per lane: x = normalised inputs of
// the lane's point (x[6] = 1 carries the first-layer bias); y = raw outputs.
// Must be reached by all 64 lanes.
__device__ __forceinline__ void mlp_wave(const FwdFrag& F, const float x[8], float y[3], int lane) {
    const bool hi = lane >= 32;
    const uint32_t w0 = pack_bf16x2(x[0], x[1]), w1 = pack_bf16x2(x[2], x[3]);
    const uint32_t w2 = pack_bf16x2(x[4], x[5]), w3 = pack_bf16x2(x[6], x[7]);
    // tile 0 = points 0..31, tile 1 = points 32..63; the partner lane l ^ 32
    // holds the other half of the inputs of the same tile column
    const uint32_t r0 = __shfl_xor(hi ? w0 : w2, 32), r1 = __shfl_xor(hi ? w1 : w3, 32);
    const s4 b0 = hi ? make_s4(r0, r1) : make_s4(w0, w1);
    const s4 b1 = hi ? make_s4(w2, w3) : make_s4(r0, r1);
    s4 h1[8], h2[8];
    const f16v o0 = forward_tile(F, b0, h1, h2);
    const f16v o1 = forward_tile(F, b1, h1, h2);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float e = __shfl_xor(o1[c], 32);
        y[c] = hi ? e : o0[c];
    }
}

// ---------------------------------------------------------------------------
// inference path (x16 products, activations chained in registers)
// ---------------------------------------------------------------------------
// Inference operands of one lane, staged in LDS once per block (all waves of
// the block read their lane's copy just before each product):
//   [0, 32)  W2 x16 A operands [mt][kb][4]     [32, 48) W3 x16 [kb][4]
//   [48, 80) b2 accumulator init [mt][16]       [80, 84) W1 x8 [mt][2]
constexpr int kLdsI2 = 0, kLdsI3 = 32, kLdsB2 = 48, kLdsW1 = 80, kLdsStride = 84;

struct InferLds {
    uint32_t w[64 * kLdsStride];
    float b3[4];
};

// Weight fragments into LDS (lane-major rows of kLdsStride words).  Element
// e = o * 64 + lane reads word(o) of that lane, so that each group of 64
// consecutive threads reads 256 contiguous bytes; all loads are issued before
// the first LDS store.  Requires blockDim.x == 256.
__device__ __forceinline__ void stage_infer_frag(InferLds& L, const uint32_t* __restrict__ frag) {
    constexpr int kIter = 64 * kLdsStride / 256;
    static_assert(64 * kLdsStride % 256 == 0, "whole iterations");
    uint32_t v[kIter];
#pragma unroll
    for (int i = 0; i < kIter; ++i) {
        const int e = i * 256 + threadIdx.x;
        const int o = e >> 6, lane = e & 63;
        int word;
        if (o < kLdsI3) word = kFragI2 + o;
        else if (o < kLdsB2) word = kFragI3 + (o - kLdsI3);
        else if (o < kLdsW1) word = kFragB2 + (o - kLdsB2);
        else word = kFragW1 + (o - kLdsW1);
        v[i] = frag[word * 64 + lane];
    }
#pragma unroll
    for (int i = 0; i < kIter; ++i) {
        const int e = i * 256 + threadIdx.x;
        L.w[(e & 63) * kLdsStride + (e >> 6)] = v[i];
    }
    if (threadIdx.x < 3) L.b3[threadIdx.x] = __uint_as_float(frag[kFragUniform + threadIdx.x]);
    __syncthreads();
}

__device__ __forceinline__ bf8v lds_bf8(const InferLds& L, int lane, int o) {
    return *reinterpret_cast<const bf8v*>(&L.w[lane * kLdsStride + o]);
}
__device__ __forceinline__ f16v lds_f16(const InferLds& L, int lane, int o) {
    return *reinterpret_cast<const f16v*>(&L.w[lane * kLdsStride + o]);
}
__device__ __forceinline__ s4 lds_w1(const InferLds& L, int lane, int mt) {
    return *reinterpret_cast<const s4*>(&L.w[lane * kLdsStride + kLdsW1 + 2 * mt]);
}

// ReLU + bf16 of accumulator registers r0..r0+7 as an x16 B operand
__device__ __forceinline__ bf8v act8(const f16v& d, int r0) {
    const u4v w = {relu_bf16x2(pack_bf16x2(d[r0], d[r0 + 1])), relu_bf16x2(pack_bf16x2(d[r0 + 2], d[r0 + 3])),
                   relu_bf16x2(pack_bf16x2(d[r0 + 4], d[r0 + 5])), relu_bf16x2(pack_bf16x2(d[r0 + 6], d[r0 + 7]))};
    return __builtin_bit_cast(bf8v, w);
}

// outputs of one 32-point tile (rows 0..2 of lanes with h = 0, without b3)
__device__ __forceinline__ f16v infer_tile(const InferLds& L, int lane, s4 xb) {
    const f16v zero = {};
    const f16v d0 = mfma(lds_w1(L, lane, 0), xb, zero), d1 = mfma(lds_w1(L, lane, 1), xb, zero);
    const bf8v h1[4] = {act8(d0, 0), act8(d0, 8), act8(d1, 0), act8(d1, 8)};
    f16v e0 = lds_f16(L, lane, kLdsB2), e1 = lds_f16(L, lane, kLdsB2 + 16);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        e0 = mfma16(lds_bf8(L, lane, kLdsI2 + kb * 4), h1[kb], e0);
        e1 = mfma16(lds_bf8(L, lane, kLdsI2 + (4 + kb) * 4), h1[kb], e1);
    }
    const bf8v h2[4] = {act8(e0, 0), act8(e0, 8), act8(e1, 0), act8(e1, 8)};
    f16v o = zero;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) o = mfma16(lds_bf8(L, lane, kLdsI3 + kb * 4), h2[kb], o);
    return o;
}

// network on the 64 points of a wave (one per lane); must be reached by all
// 64 lanes
__device__ __forceinline__ void mlp_infer(const InferLds& L, const float x[8], float y[3], int lane) {
    // compiler-only barrier: keeps the operand loads from LDS here instead of
    // letting them be hoisted out of the point loop into (many) registers
    __asm__ volatile("" ::: "memory");
    const bool hi = lane >= 32;
    const uint32_t w0 = pack_bf16x2(x[0], x[1]), w1 = pack_bf16x2(x[2], x[3]);
    const uint32_t w2 = pack_bf16x2(x[4], x[5]), w3 = pack_bf16x2(x[6], x[7]);
    const uint32_t r0 = __shfl_xor(hi ? w0 : w2, 32), r1 = __shfl_xor(hi ? w1 : w3, 32);
    const f16v o0 = infer_tile(L, lane, hi ? make_s4(r0, r1) : make_s4(w0, w1));
    const f16v o1 = infer_tile(L, lane, hi ? make_s4(w2, w3) : make_s4(r0, r1));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float e = __shfl_xor(o1[c], 32);
        y[c] = (hi ? e : o0[c]) + L.b3[c];
    }
}

// ---------------------------------------------------------------------------
// fragment packing from the float32 master parameters (one wave)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float w1ext(const float* P, int r, int k) {
    return k < 6 ? P[kOffW1 + r * 6 + k] : (k == 6 ? P[kOffB1 + r] : 0.0f);
}

__global__ __launch_bounds__(64) void pack_kernel(const float* __restrict__ P, uint32_t* __restrict__ frag) {
    const int lane = threadIdx.x, h = lane >> 5, j = lane & 31;
    auto put = [&](int word, float a, float b) { frag[word * 64 + lane] = pack_bf16x2(a, b); };
    for (int mt = 0; mt < 2; ++mt) {
        const int row = mt * 32 + j;
        put(kFragW1 + 2 * mt, w1ext(P, row, 4 * h), w1ext(P, row, 4 * h + 1));
        put(kFragW1 + 2 * mt + 1, w1ext(P, row, 4 * h + 2), w1ext(P, row, 4 * h + 3));
        for (int kb = 0; kb < 8; ++kb) {
            const int col = kb * 8 + 4 * h;
            const float* w = P + kOffW2 + row * 64 + col;
            put(kFragW2 + 2 * (mt * 8 + kb), w[0], w[1]);
            put(kFragW2 + 2 * (mt * 8 + kb) + 1, w[2], w[3]);
            // transposed W2: A[i = row][k = col + c] = W2[col + c][row]
            const float* t = P + kOffW2 + col * 64 + row;
            put(kFragW2T + 2 * (mt * 8 + kb), t[0], t[64]);
            put(kFragW2T + 2 * (mt * 8 + kb) + 1, t[128], t[192]);
        }
        // transposed W3: A[i = hidden row][k = output 4h + c]
        float v[4];
        for (int c = 0; c < 4; ++c) v[c] = (4 * h + c < 3) ? P[kOffW3 + (4 * h + c) * 64 + row] : 0.0f;
        put(kFragW3T + 2 * mt, v[0], v[1]);
        put(kFragW3T + 2 * mt + 1, v[2], v[3]);
        for (int r = 0; r < 16; ++r) {
            const int i = mt * 32 + (r & 3) + 4 * h + 8 * (r >> 2);
            frag[(kFragB2 + mt * 16 + r) * 64 + lane] = __float_as_uint(P[kOffB2 + i]);
        }
    }
    for (int kb = 0; kb < 8; ++kb) {
        const int col = kb * 8 + 4 * h;
        float v[4];
        for (int c = 0; c < 4; ++c) v[c] = (j < 3) ? P[kOffW3 + j * 64 + col + c] : 0.0f;
        put(kFragW3 + 2 * kb, v[0], v[1]);
        put(kFragW3 + 2 * kb + 1, v[2], v[3]);
    }
    for (int r = 0; r < 16; ++r) {
        const int i = (r & 3) + 4 * h + 8 * (r >> 2);
        frag[(kFragB3 + r) * 64 + lane] = __float_as_uint(i < 3 ? P[kOffB3 + i] : 0.0f);
    }
    // inference operands with the chained k order
    for (int kb = 0; kb < 4; ++kb) {
        for (int pr = 0; pr < 4; ++pr) {
            const int f0 = chained_feature(kb, h, 2 * pr), f1 = chained_feature(kb, h, 2 * pr + 1);
            for (int mt = 0; mt < 2; ++mt) {
                const int row = mt * 32 + j;
                put(kFragI2 + (mt * 4 + kb) * 4 + pr, P[kOffW2 + row * 64 + f0], P[kOffW2 + row * 64 + f1]);
            }
            put(kFragI3 + kb * 4 + pr, j < 3 ? P[kOffW3 + j * 64 + f0] : 0.0f, j < 3 ? P[kOffW3 + j * 64 + f1] : 0.0f);
        }
    }
    if (lane < 3) frag[kFragUniform + lane] = __float_as_uint(P[kOffB3 + lane]);
}

hipError_t mlp_pack(const MlpState& s, hipStream_t st) {
    hipLaunchKernelGGL(pack_kernel, dim3(1), dim3(64), 0, st, s.master, s.frag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched inference on raw inputs X[B][6] -> deltas Y[B][3] (outputs x out_scale)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void normalise(const MlpNorm& n, const float raw[6], float x[8]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) x[k] = (raw[k] - n.in_mean[k]) * n.in_inv_scale[k];
    x[6] = 1.0f;
    x[7] = 0.0f;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void forward_kernel(const float* __restrict__ X, int64_t B,
                                                     float* __restrict__ Y, const uint32_t* __restrict__ frag,
                                                     MlpNorm nrm) {
    __shared__ InferLds L;
    stage_infer_frag(L, frag);
    const int lane = threadIdx.x & 63;
    const int64_t n_chunks = (B + 63) >> 6;
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t chunk = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; chunk < n_chunks;
         chunk += n_waves) {
        const int64_t p = chunk * 64 + lane;
        const bool valid = p < B;
        float raw[6], x[8], y[3];
#pragma unroll
        for (int k = 0; k < 6; ++k) raw[k] = valid ? X[p * 6 + k] : nrm.in_mean[k];
        normalise(nrm, raw, x);
        mlp_infer(L, x, y, lane);
        if (valid) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Y[p * 3 + c] = y[c] * nrm.out_scale[c];
        }
    }
}

hipError_t mlp_forward(const MlpState& s, const float* X, int64_t B, float* Y, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    const int64_t chunks = (B + 63) / 64;
    const int64_t blocks = chunks < 1024 ? (chunks + 3) / 4 : 256;
    hipLaunchKernelGGL(forward_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, B, Y, s.frag, s.norm);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// training: one wave per block; per 64-sample chunk a forward and backward
// pass in registers, then the weight gradients as products over the chunk's
// samples from LDS copies (features x samples, bf16) of X, H1, H2, dY, dH2,
// dH1.  Each wave writes its partial gradient; a second kernel sums the
// partials in wave order (deterministic).  Loss: 0.5/B sum ||f(x) - y/s||^2.
// ---------------------------------------------------------------------------
constexpr int kMaxTrainWaves = 1024;

struct TrainLds {
    uint16_t X[8][64];
    uint16_t H1[64][64];
    uint16_t H2[64][64];
    uint16_t dH2[64][64];
    uint16_t dH1[64][64];
    uint16_t dY[8][64];
};

__device__ __forceinline__ s4 lds_s4(const uint16_t* row, int col) {
    return *reinterpret_cast<const s4*>(row + col);
}

__device__ __forceinline__ void store_cols(uint16_t (*M)[64], int row0, int col, s4 v) {
#pragma unroll
    for (int c = 0; c < 4; ++c) M[row0 + c][col] = (uint16_t)v[c];
}

__global__ __launch_bounds__(64) void train_kernel(const float* __restrict__ X, const float* __restrict__ Y, int64_t B,
                                                  const uint32_t* __restrict__ frag, MlpNorm nrm,
                                                  float* __restrict__ partial) {
    __shared__ TrainLds L;
    const int lane = threadIdx.x, h = lane >> 5, j = lane & 31;
    const int wave = blockIdx.x, n_waves = gridDim.x;
    FwdFrag F;
    load_fwd_frag(F, frag, lane);
    s4 w3t[2], w2t[2][8];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        w3t[mt] = frag_s4(frag, kFragW3T + 2 * mt, lane);
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) w2t[mt][kb] = frag_s4(frag, kFragW2T + 2 * (mt * 8 + kb), lane);
    }
    const f16v zero = {};
    f16v gW1[2] = {zero, zero}, gW2[2][2] = {{zero, zero}, {zero, zero}}, gW3[2] = {zero, zero};
    float gb2 = 0.0f, gb3 = 0.0f, lsum = 0.0f;
    const float invB = 1.0f / (float)B;
    const int64_t n_chunks = (B + 63) >> 6;

    for (int64_t chunk = wave; chunk < n_chunks; chunk += n_waves) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int col = 32 * t + j;
            const int64_t p = chunk * 64 + col;
            const bool valid = p < B;
            float xin[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int k = 4 * h + c;
                float v = 0.0f;
                if (valid) v = k < 6 ? (X[p * 6 + k] - nrm.in_mean[k]) * nrm.in_inv_scale[k] : (k == 6 ? 1.0f : 0.0f);
                xin[c] = v;
            }
            const s4 xb = make_s4(pack_bf16x2(xin[0], xin[1]), pack_bf16x2(xin[2], xin[3]));
            store_cols(L.X, 4 * h, col, xb);
            s4 h1[8], h2[8];
            const f16v o = forward_tile(F, xb, h1, h2);
#pragma unroll
            for (int kb = 0; kb < 8; ++kb) {
                store_cols(L.H1, kb * 8 + 4 * h, col, h1[kb]);
                store_cols(L.H2, kb * 8 + 4 * h, col, h2[kb]);
            }
            // residual and output gradient on the lanes that hold the outputs
            float dy[3] = {0.0f, 0.0f, 0.0f};
            if (h == 0 && valid) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float r = o[c] - Y[p * 3 + c] / nrm.out_scale[c];
                    lsum = fmaf(0.5f * r, r, lsum);
                    dy[c] = r * invB;
                }
            }
            const s4 dyb = make_s4(pack_bf16x2(dy[0], dy[1]), pack_bf16x2(dy[2], 0.0f));
            store_cols(L.dY, 4 * h, col, dyb);
            // dH2^T = W3^T dY^T, masked by H2 > 0
            s4 dh2[8];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const f16v d = mfma(w3t[mt], dyb, zero);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const s4 m = h2[mt * 4 + q];
                    float v[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) v[c] = (m[c] > 0) ? d[4 * q + c] : 0.0f;
                    dh2[mt * 4 + q] = make_s4(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
                    store_cols(L.dH2, mt * 32 + 8 * q + 4 * h, col, dh2[mt * 4 + q]);
                }
            }
            // dH1^T = W2^T dH2^T, masked by H1 > 0
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                f16v acc = zero;
#pragma unroll
                for (int kb = 0; kb < 8; ++kb) acc = mfma(w2t[mt][kb], dh2[kb], acc);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const s4 m = h1[mt * 4 + q];
                    float v[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) v[c] = (m[c] > 0) ? acc[4 * q + c] : 0.0f;
                    store_cols(L.dH1, mt * 32 + 8 * q + 4 * h,
                               col, make_s4(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3])));
                }
            }
        }
        __syncthreads();
        // weight gradients: sums over the 64 samples of the chunk
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
            const int c0 = kb * 8 + 4 * h;
            const s4 xB = j < 8 ? lds_s4(L.X[j & 7], c0) : s4{0, 0, 0, 0};
            const s4 dyA = j < 3 ? lds_s4(L.dY[j & 7], c0) : s4{0, 0, 0, 0};
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const s4 a2 = lds_s4(L.dH2[mt * 32 + j], c0);
                const s4 a1 = lds_s4(L.dH1[mt * 32 + j], c0);
                gW1[mt] = mfma(a1, xB, gW1[mt]);
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) gW2[mt][nt] = mfma(a2, lds_s4(L.H1[nt * 32 + j], c0), gW2[mt][nt]);
            }
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) gW3[nt] = mfma(dyA, lds_s4(L.H2[nt * 32 + j], c0), gW3[nt]);
        }
        // bias gradients: row sums (lane l owns hidden row l and output row l < 3)
        {
            float s2 = 0.0f, s3 = 0.0f;
            for (int c = 0; c < 64; ++c) {
                s2 += bf16_bits_to_float(L.dH2[lane][c]);
                if (lane < 3) s3 += bf16_bits_to_float(L.dY[lane][c]);
            }
            gb2 += s2;
            gb3 += s3;
        }
        __syncthreads();
    }
    // partial gradient of this wave
    float* P = partial + (int64_t)wave * (kMlpParams + 1);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = mt * 32 + (r & 3) + 4 * h + 8 * (r >> 2);
            if (j < 6) P[kOffW1 + i * 6 + j] = gW1[mt][r];
            else if (j == 6) P[kOffB1 + i] = gW1[mt][r];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) P[kOffW2 + i * 64 + nt * 32 + j] = gW2[mt][nt][r];
        }
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int o = (r & 3) + 4 * h + 8 * (r >> 2);
            if (o < 3) P[kOffW3 + o * 64 + nt * 32 + j] = gW3[nt][r];
        }
    }
    P[kOffB2 + lane] = gb2;
    if (lane < 3) P[kOffB3 + lane] = gb3;
    // loss: wave sum in a fixed order
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off);
    if (lane == 0) P[kMlpParams] = lsum;
}

__global__ __launch_bounds__(256) void reduce_kernel(const float* __restrict__ partial, int n_waves,
                                                    float* __restrict__ grad, float* __restrict__ loss,
                                                    float invB) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > kMlpParams) return;
    float s = 0.0f;
    for (int w = 0; w < n_waves; ++w) s += partial[(int64_t)w * (kMlpParams + 1) + p];
    if (p < kMlpParams) grad[p] = s;
    else loss[0] = s * invB;
}

hipError_t mlp_grad(MlpState& s, const float* X, const float* Y, int64_t B, float* grad, float* loss,
                    hipStream_t st) {
    const int64_t chunks = (B + 63) / 64;
    const int waves = (int)(chunks < kMaxTrainWaves ? chunks : kMaxTrainWaves);
    hipLaunchKernelGGL(train_kernel, dim3(waves), dim3(64), 0, st, X, Y, B, s.frag, s.norm, s.partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_kernel, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, st, s.partial, waves, grad,
                       loss, 1.0f / (float)B);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                                  const float* __restrict__ g, float lr, float bc1, float bc2) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kMlpParams) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.0f - b1) * gi;
    const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    w[p] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

hipError_t mlp_adam(MlpState& s, float lr, hipStream_t st) {
    s.adam_t += 1;
    const float bc1 = 1.0f - powf(0.9f, (float)s.adam_t), bc2 = 1.0f - powf(0.999f, (float)s.adam_t);
    hipLaunchKernelGGL(adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, s.master, s.adam_m, s.adam_v,
                       s.grad, lr, bc1, bc2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return mlp_pack(s, st);
}

// ---------------------------------------------------------------------------
// Surrogate mode inside the fused launches.  A launch covers up to 64 steps
// (a whole number of network blocks of Ks steps) with the launch
// certificates, wave flags and slot kernels of the plain path.  A wave that
// steps decides block by block: if every one of its active points passes
// the error indicator, the block is one explicit step of Ks dt (rates at the
// block-start temperature, the Appendix A start-up forms included), the
// network's correction towards Ks plain steps where an increment exceeds
// kNetMinIncrement, and the correction g at the block-end temperature;
// otherwise the wave takes the Ks plain steps, evaluating the temperature
// at each.  The network runs in a second kernel: a wave that needs it at
// block j leaves its state at the start of block j in a record and stops,
// and the resume kernel (weights staged in LDS) carries on from there.  So
// the fused kernels keep the plain path's register budget.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool needs_plain(float T0, float TK, const MlpNorm& n) {
    const float lo = fminf(T0, TK), hi = fmaxf(T0, TK);
    const bool cold = hi < n.T_cold;
    const bool hot = lo >= n.T_hot_lo && hi <= n.T_hot_hi;
    return !(cold || hot) || fabsf(TK - T0) > n.dT_max;
}

// A point at its martensite formation front: within kFrontProbe of the lower
// block-end temperature the formation law would raise alpha_m, so a dip of the
// temperature inside the block would form martensite the block ends miss.
constexpr float kFrontProbe = 5.0f;  // [K]
// The network corrects one explicit step of Ks dt towards Ks plain steps.
// The two differ by the change of the rates over the block times Ks dt, at
// most about the increment itself, so increments of at most 2^-20 (about
// 1e-6) in both fractions are taken as they are.  Away from the laser these
// are the slow low-temperature rates, e.g. the tempering of martensite.
constexpr float kNetMinIncrement = 0x1p-20f;
constexpr int kProbeEvery = 8;  // probe spacing inside longer blocks [steps]
__device__ __forceinline__ bool formation_front(float T0, float TK, float a, float m) {
    const float Tlo = fminf(T0, TK) - kFrontProbe;
    return Tlo < kTamStart && am0_eq(Tlo) * (kXmax - a) * (1.0f / kXmax) > m;
}

// a wave's state at the start of a block, handed to the resume kernel
struct SurrogateRecord {
    int64_t wave;
    int32_t block;
    int32_t cold;
    int32_t launch;  // the launch of the call (persistent form; the launch form does not read it)
    int32_t pad;
    float a[kWave], m[kWave], alo[kWave], mlo[kWave], Tn[kWave];
};

// What a wave does with a block whose increments need the network.
enum { kNetStop = 0, kNetRun = 1, kNetPlain = 2 };

// Blocks j0 .. of a launch of Kl steps for the calling lane's point (state
// in registers: (a, alo), (m, mlo) compensated pairs, Tn the temperature at
// the start of block j0).  NET: kNetStop returns the block at which the
// network is needed (state unchanged from that block's start); kNetRun
// evaluates it (all 64 lanes; L: staged weights); kNetPlain takes the plain
// steps instead.  Returns -1 when every block was taken.  frozen_nb > 1 (a
// cold wave from block 0, whose blocks all take the block update): if block
// 0 left the fractions' stored values as they were over frozen_nb blocks
// (frozen_part), every later block repeats it, and the blocks stop there
// with a, m as on entry and alo = mlo = 0 (returns -2).
template <int W, int NET>
__device__ __forceinline__ int surrogate_blocks(const PointGeom& pg, const SrcRec* __restrict__ tab, int Kl, int Ks,
                                                float dt, const ScanArgs& sa, const MlpNorm& nrm,
                                                const InferLds* L, bool act, bool cold, int gi, int gj, int gk, int j0,
                                                float& a, float& m, float& alo, float& mlo, float& Tn,
                                                int frozen_nb = 0) {
    const float T0c = fminf(sa.T0, sa.Tclamp);
    const float a0 = a, m0 = m;
    const int nb = (Kl + Ks - 1) / Ks;
    float xeq_n = alpha_eq(Tn);
    for (int j = j0; j < nb; ++j) {
        const int s0 = j * Ks, Kb = min(Ks, Kl - s0);
        const SrcRec* tb = tab + s0 * W;
        const float TK = cold ? T0c : scan_temperature<W>(tb + Kb * W, gi, gj, gk, sa.T0, sa.Tclamp, pg.r2min, pg.roff);
        // the indicator, point by point; a partial block (the end of a
        // call) takes the plain steps
        bool plain = Kb < Ks || needs_plain(Tn, TK, nrm);
        if (act && !plain && !cold && formation_front(Tn, TK, a, m)) {
            // martensite forms at the lowest temperature of the block: a dip
            // below both ends needs the plain steps.  Probed at the block
            // middle and every kProbeEvery steps.
            const float Tlo = fminf(Tn, TK);
            plain = scan_temperature<W>(tb + (Kb / 2) * W, gi, gj, gk, sa.T0, sa.Tclamp, pg.r2min, pg.roff) < Tlo;
            for (int s = kProbeEvery; s < Kb && !plain; s += kProbeEvery) {
                if (s == Kb / 2) continue;
                plain = scan_temperature<W>(tb + s * W, gi, gj, gk, sa.T0, sa.Tclamp, pg.r2min, pg.roff) < Tlo;
            }
        }
        const bool rest = !act || at_rest(a, m, Tn, TK);
        float da = 0.0f, dm = 0.0f;
        bool need = false;
        if (!plain && !rest) {
            diffusive_increment(a, m, Tn, xeq_n, dt * (float)Kb, da, dm);
            need = fmaxf(fabsf(da), fabsf(dm)) > kNetMinIncrement;
        }
        const bool wave_plain = __ballot(act && plain) != 0;
        const bool wave_net = !wave_plain && __ballot(need) != 0;
        if (NET == kNetStop && wave_net) return j;
        if (wave_plain || (NET == kNetPlain && wave_net)) {
            // the Kb plain steps; the last temperature is TK
            for (int s = 0; s < Kb; ++s) {
                const float Tn1 = (s + 1 == Kb) ? TK
                                  : cold        ? T0c
                                                : scan_temperature<W>(tb + (s + 1) * W, gi, gj, gk, sa.T0, sa.Tclamp,
                                                                      pg.r2min, pg.roff);
                const float xeq_n1 = alpha_eq(Tn1);
                explicit_step<true>(a, m, alo, mlo, Tn, xeq_n, Tn1, xeq_n1, dt);
                Tn = Tn1;
                xeq_n = xeq_n1;
            }
            continue;
        }
        float ra = 0.0f, rm = 0.0f;
        if (NET == kNetRun && wave_net) {
            // inputs (T_n, T_K, ln dt, beta, alpha_s, alpha_m) at the block start
            const float raw[6] = {Tn, TK, logf(dt), solid_fraction(Tn) - a - m, a, m};
            float x[8], y[3];
            normalise(nrm, raw, x);
            mlp_infer(*L, x, y, threadIdx.x & (kWave - 1));
            if (need) {
                ra = y[0] * nrm.out_scale[0];
                rm = y[1] * nrm.out_scale[1];
            }
        }
        const float xeq_K = alpha_eq(TK);
        if (!rest) {
            float at, mt;
            two_sum(a, alo + (da + ra), at, alo);
            two_sum(m, mlo + (dm + rm), mt, mlo);
            const float a_before = at, m_before = mt;
            correct(TK, xeq_K, at, mt);
            if (at != a_before) alo = 0.0f;
            if (mt != m_before) mlo = 0.0f;
            a = at;
            m = mt;
        }
        Tn = TK;
        xeq_n = xeq_K;
        if (frozen_nb > 1 && j == 0 &&
            __ballot(act && !(frozen_part(a0, a, alo, frozen_nb) && frozen_part(m0, m, mlo, frozen_nb))) == 0) {
            a = a0;
            m = m0;
            alo = 0.0f;
            mlo = 0.0f;
            return -2;
        }
    }
    return -1;
}

// the end of a wave's launch: its state, beta in the last launch of a call,
// its rest flag
__device__ __forceinline__ void surrogate_store(const EnvSet& env, int64_t wv, bool act, int64_t local, float a,
                                                float m, float alo, float mlo, float Tn, float* __restrict__ beta,
                                                float* __restrict__ as, float* __restrict__ am) {
    const float af = a + alo, mf = m + mlo;
    if (act) {
        as[local] = af;
        am[local] = mf;
        if (beta) beta[local] = solid_fraction(Tn) - af - mf;
    }
    record_rest(env, wv, act, af, mf);
}

// One surrogate launch of a wave on its register state: still and cold
// waves as in the plain fused kernel, then the network blocks.  A cold wave
// whose blocks all take the block update (whole blocks, and the indicator
// passes at T0) stops after its first block if that block left the stored
// fractions as they were (frozen: every block starts from the same high
// parts at T0 and repeats the first, so the launch would store the loaded
// values).  a, m: the fractions as loaded; returns 0 (still: a, m unchanged,
// Tn = T0), 1 (frozen: the same, with alo = mlo = 0), 2 (done: hi parts a, m
// and lo parts alo, mlo at the end of the launch, Tn its last temperature)
// or, with NET == kNetStop, 3: block j needs the network, and a, m, alo,
// mlo, Tn hold the state at that block's start (cold: whether the wave is
// cold in this launch).
template <int W, int NET>
__device__ __forceinline__ int surrogate_launch(const PointGeom& pg, const SrcRec* __restrict__ tab, const EnvSet& env,
                                                int64_t wv, int Kl, int Ks, float dt, const ScanArgs& sa,
                                                const MlpNorm& nrm, const InferLds* L, bool act, int gi, int gj,
                                                int gk, float& a, float& m, float& alo, float& mlo, float& Tn,
                                                bool& cold_out, int& j) {
    const float T0c = fminf(sa.T0, sa.Tclamp);
    alo = 0.0f;
    mlo = 0.0f;
    const float rlim2 = envelope_radius2(pg);
    const bool tried = wave_may_rest(env, act, a, m, T0c);
    bool still = tried && (wave_box_below(env, wv) ||
                           wave_below(env.rec, env.n, act, gi, gj, gk, rlim2, T0c, kRestBelow));
    const bool cold = still || (!tried && wave_cold(env.rec, env.n, act, gi, gj, gk, rlim2));
    Tn = cold ? T0c : scan_temperature<W>(tab, gi, gj, gk, sa.T0, sa.Tclamp, pg.r2min, pg.roff);
    still = still || (cold && T0c < Const<float>::TasEnd && __ballot(act && !rest_bits(a, m)) == 0);
    if (env.stats) count_wave(env, act, still, cold);
    cold_out = cold;
    if (still) return 0;  // its fractions are those in memory
    if (!cold) __builtin_amdgcn_s_setprio(3);  // as in plain_launch
    const int nb = Kl / Ks;
    const int frozen_nb = (cold && nb > 1 && nb * Ks == Kl && !needs_plain(T0c, T0c, nrm)) ? nb : 0;
    j = surrogate_blocks<W, NET>(pg, tab, Kl, Ks, dt, sa, nrm, L, act, cold, gi, gj, gk, 0, a, m, alo, mlo, Tn,
                                 frozen_nb);
    __builtin_amdgcn_s_setprio(0);
    return j >= 0 ? 3 : j == -2 ? 1 : 2;
}

// a wave's state at the start of block j of launch l, for the resume kernels
// (written by every lane: no branch on the lane)
__device__ __forceinline__ void write_record(SurrogateRecord& r, int64_t wv, int j, bool cold, int64_t l, float a,
                                             float m, float alo, float mlo, float Tn) {
    const int lane = threadIdx.x & (kWave - 1);
    r.wave = wv;
    r.block = j;
    r.cold = cold ? 1 : 0;
    r.launch = (int32_t)l;
    r.a[lane] = a;
    r.m[lane] = m;
    r.alo[lane] = alo;
    r.mlo[lane] = mlo;
    r.Tn[lane] = Tn;
}

// the body of a fused surrogate launch for wave wv (points g = 64 wv + lane)
template <int W>
__device__ __forceinline__ void surrogate_fused_body(const PointGeom& pg, const SrcRec* __restrict__ tab,
                                                     const EnvSet& env, int Kl, int Ks, float dt, const ScanArgs& sa,
                                                     const MlpNorm& nrm, float* __restrict__ beta,
                                                     float* __restrict__ as, float* __restrict__ am,
                                                     SurrogateRecord* __restrict__ recs, unsigned* __restrict__ n_recs,
                                                     int64_t cap, int64_t g, int64_t wv) {
    bool act = g < pg.count;
    int gi, gj, gk;
    const int64_t local = point_at(pg, act ? g : 0, gi, gj, gk);
    act = act && gk >= pg.k0;
    float a = act ? as[local] : 0.0f, m = act ? am[local] : 0.0f, alo, mlo, Tn;
    bool cold;
    int j = -1;
    const int r = surrogate_launch<W, kNetStop>(pg, tab, env, wv, Kl, Ks, dt, sa, nrm, nullptr, act, gi, gj, gk, a, m,
                                                alo, mlo, Tn, cold, j);
    if (r == 0 || r == 1) {  // still or frozen: its fractions are those in memory
        if (act && beta) beta[local] = solid_fraction(Tn) - a - m;
        record_rest(env, wv, act, a, m);
        return;
    }
    if (r == 3) {
        const unsigned slot =
            __builtin_amdgcn_readfirstlane(atomicAdd(n_recs, (threadIdx.x & (kWave - 1)) == 0 ? 1u : 0u));
        if ((int64_t)slot < cap) {
            write_record(recs[slot], wv, j, cold, 0, a, m, alo, mlo, Tn);
            return;  // the resume kernel takes the wave from block j
        }
        // no room for the record: this wave takes plain steps where the network would act
        surrogate_blocks<W, kNetPlain>(pg, tab, Kl, Ks, dt, sa, nrm, nullptr, act, cold, gi, gj, gk, j, a, m, alo, mlo,
                                       Tn);
    }
    surrogate_store(env, wv, act, local, a, m, alo, mlo, Tn, beta, as, am);
}

template <int W>
__global__ __launch_bounds__(kFusedBlock) void fused_surrogate_kernel(PointGeom pg, const SrcRec* __restrict__ tab,
                                                                      EnvSet env, int Kl, int Ks, float dt,
                                                                      ScanArgs sa, MlpNorm nrm,
                                                                      float* __restrict__ beta, float* __restrict__ as,
                                                                      float* __restrict__ am,
                                                                      SurrogateRecord* __restrict__ recs,
                                                                      unsigned* __restrict__ n_recs, int64_t cap) {
    const int64_t wv = fused_wave();
    const int64_t g = (int64_t)blockIdx.x * kFusedBlock + threadIdx.x;
    if (wave_flag_still(env, wv)) {
        still_wave_beta(pg, fminf(sa.T0, sa.Tclamp), beta, g);
        if (env.stats && (threadIdx.x & (kWave - 1)) == 0) atomicAdd(env.stats + kStatFlagged, 1ull);
        return;
    }
    surrogate_fused_body<W>(pg, tab, env, Kl, Ks, dt, sa, nrm, beta, as, am, recs, n_recs, cap, g, wv);
}

// The waves that stopped for the network: a persistent grid, each wave one
// record at a time, from the recorded block to the end of the launch with
// the network evaluated where it is needed.  Zeroes the other record counter
// for the next launch.
template <int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void surrogate_resume_kernel(
    PointGeom pg, const SrcRec* __restrict__ tab, EnvSet env, int Kl, int Ks, float dt, ScanArgs sa, MlpNorm nrm,
    float* __restrict__ beta, float* __restrict__ as, float* __restrict__ am, const SurrogateRecord* __restrict__ recs,
    const unsigned* __restrict__ n_recs, unsigned* __restrict__ n_recs_next, int64_t cap, const uint32_t* __restrict__ frag) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_recs_next = 0u;
    const int64_t count = min((int64_t)*n_recs, cap);
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    if ((int64_t)blockIdx.x * (blockDim.x >> 6) >= count) return;  // no record for this block (uniform)
    __shared__ InferLds L;
    stage_infer_frag(L, frag);
    const int lane = threadIdx.x & (kWave - 1);
    for (int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; q < count; q += n_waves) {
        const SurrogateRecord& r = recs[q];
        const int64_t wv = r.wave, g = wv * kWave + lane;
        bool act = g < pg.count;
        int gi, gj, gk;
        const int64_t local = point_at(pg, act ? g : 0, gi, gj, gk);
        act = act && gk >= pg.k0;
        float a = r.a[lane], m = r.m[lane], alo = r.alo[lane], mlo = r.mlo[lane], Tn = r.Tn[lane];
        surrogate_blocks<W, kNetRun>(pg, tab, Kl, Ks, dt, sa, nrm, &L, act, r.cold != 0, gi, gj, gk, r.block, a, m, alo,
                                     mlo, Tn);
        surrogate_store(env, wv, act, local, a, m, alo, mlo, Tn, beta, as, am);
    }
}

// ---------------------------------------------------------------------------
// SURROGATE calls in the persistent form of the plain path (see
// fused_plain_call_kernel): per chunk of launches the list pass,
// fused_surrogate_call_kernel and surrogate_resume_call_kernel.  The call
// kernel runs each listed wave through the chunk's launches on registers
// without the network; a wave with a block that needs the network records
// its state at that block's start and the launch, and leaves the rest of the
// chunk to the resume kernel, which evaluates the network there and runs the
// wave's remaining launches of the chunk, the network wherever it is needed.
// What each wave computes is what the launch-by-launch form computes.  No
// branch on the lane inside the kernels' loops (see fused_call).
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kCallBlock) void fused_surrogate_call_kernel(
    PointGeom pg, const SrcRec* __restrict__ tab, const EnvRec* __restrict__ env, const int32_t* __restrict__ env_fc,
    const uint8_t* __restrict__ below, uint8_t* __restrict__ rest, int64_t n_waves, int64_t l0, int64_t nl, int Kl,
    int Ks, int64_t n_steps, float dt, ScanArgs sa, MlpNorm nrm, float* __restrict__ beta, float* __restrict__ as,
    float* __restrict__ am, const uint32_t* __restrict__ cand, const unsigned* __restrict__ counts,
    unsigned* __restrict__ next, unsigned long long* __restrict__ stats, SurrogateRecord* __restrict__ recs,
    unsigned* __restrict__ n_recs, int64_t cap) {
    const float T0c = fminf(sa.T0, sa.Tclamp);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t n_list = counts[0];
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
        bool rest_w = l0 == 0 ? __ballot(act && !rest_bits(a, m)) == 0 : rest[w] != 0;
        bool changed = false, flagged = false, parked = false;
        uint64_t bm = 0;
        int64_t lb = l0 - kWave;
        for (int64_t l = l0; l < l0 + nl; ++l) {
            const uint8_t* bl = below + (l - l0) * n_waves;
            if (l - lb >= kWave) {  // (uniform) lane i loads launch l + i's flag
                lb = l;
                bm = __ballot(l + lane < l0 + nl && below[(l - l0 + lane) * n_waves + w] != 0);
            }
            flagged = rest_w && ((bm >> (l - lb)) & 1);
            if (flagged) {
                if (stats) atomicAdd(stats + kStatFlagged, lane == 0 ? 1ull : 0ull);
                continue;
            }
            const int64_t s0 = l * Kl;
            const int Kb = (int)min((int64_t)Kl, n_steps - s0);
            const EnvSet es{env + env_fc[2 * l], env_fc[2 * l + 1], bl, nullptr, n_waves, 0, stats,
                            nullptr, nullptr, nullptr};
            float alo, mlo, Tn;
            bool cold;
            int j = -1;
            int r = surrogate_launch<W, kNetStop>(pg, tab + s0 * W, es, w, Kb, Ks, dt, sa, nrm, nullptr, act, gi, gj,
                                                  gk, a, m, alo, mlo, Tn, cold, j);
            if (r == 3) {
                const unsigned slot = __builtin_amdgcn_readfirstlane(atomicAdd(n_recs, lane == 0 ? 1u : 0u));
                if ((int64_t)slot < cap) {
                    write_record(recs[slot], w, j, cold, l, a, m, alo, mlo, Tn);
                    parked = true;  // the resume kernel takes the wave from block j of launch l
                    break;
                }
                // no room for the record: plain steps where the network would act
                surrogate_blocks<W, kNetPlain>(pg, tab + s0 * W, Kb, Ks, dt, sa, nrm, nullptr, act, cold, gi, gj, gk,
                                               j, a, m, alo, mlo, Tn);
                r = 2;
            }
            if (r == 2) {  // a still or frozen wave's fractions are those in memory
                a += alo;
                m += mlo;
                changed = true;
            }
            af = a;
            mf = m;
            Tc = Tn;
            rest_w = __ballot(act && !rest_bits(af, mf)) == 0;
        }
        if (!parked) {
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
}

template <int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void surrogate_resume_call_kernel(
    PointGeom pg, const SrcRec* __restrict__ tab, const EnvRec* __restrict__ env, const int32_t* __restrict__ env_fc,
    const uint8_t* __restrict__ below, uint8_t* __restrict__ rest, int64_t n_waves, int64_t l0, int64_t nl, int Kl,
    int Ks, int64_t n_steps, float dt, ScanArgs sa, MlpNorm nrm, float* __restrict__ beta, float* __restrict__ as,
    float* __restrict__ am, const SurrogateRecord* __restrict__ recs, const unsigned* __restrict__ n_recs, int64_t cap,
    const uint32_t* __restrict__ frag, unsigned long long* __restrict__ stats) {
    const int64_t count = min((int64_t)*n_recs, cap);
    const int64_t n_grid = (int64_t)gridDim.x * (blockDim.x >> 6);
    if ((int64_t)blockIdx.x * (blockDim.x >> 6) >= count) return;  // no record for this block (uniform)
    __shared__ InferLds L;
    stage_infer_frag(L, frag);
    const float T0c = fminf(sa.T0, sa.Tclamp);
    const int lane = threadIdx.x & (kWave - 1);
    for (int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; q < count; q += n_grid) {
        const SurrogateRecord& r = recs[q];
        const int64_t w = r.wave, lp = r.launch, g = w * kWave + lane;
        bool act = g < pg.count;
        int gi, gj, gk;
        const int64_t local = point_at(pg, act ? g : 0, gi, gj, gk);
        act = act && gk >= pg.k0;
        float a = r.a[lane], m = r.m[lane], alo = r.alo[lane], mlo = r.mlo[lane], Tn = r.Tn[lane];
        // the recorded launch from its block, with the network
        int64_t s0 = lp * Kl;
        int Kb = (int)min((int64_t)Kl, n_steps - s0);
        surrogate_blocks<W, kNetRun>(pg, tab + s0 * W, Kb, Ks, dt, sa, nrm, &L, act, r.cold != 0, gi, gj, gk, r.block, a,
                                     m, alo, mlo, Tn);
        a += alo;
        m += mlo;
        float af = a, mf = m, Tc = Tn;
        bool rest_w = __ballot(act && !rest_bits(af, mf)) == 0, flagged = false;
        // the chunk's remaining launches
        uint64_t bm = 0;
        int64_t lb = lp + 1 - kWave;
        for (int64_t l = lp + 1; l < l0 + nl; ++l) {
            const uint8_t* bl = below + (l - l0) * n_waves;
            if (l - lb >= kWave) {
                lb = l;
                bm = __ballot(l + lane < l0 + nl && below[(l - l0 + lane) * n_waves + w] != 0);
            }
            flagged = rest_w && ((bm >> (l - lb)) & 1);
            if (flagged) {
                if (stats) atomicAdd(stats + kStatFlagged, lane == 0 ? 1ull : 0ull);
                continue;
            }
            s0 = l * Kl;
            Kb = (int)min((int64_t)Kl, n_steps - s0);
            const EnvSet es{env + env_fc[2 * l], env_fc[2 * l + 1], bl, nullptr, n_waves, 0, stats,
                            nullptr, nullptr, nullptr};
            bool cold;
            int j = -1;
            if (surrogate_launch<W, kNetRun>(pg, tab + s0 * W, es, w, Kb, Ks, dt, sa, nrm, &L, act, gi, gj, gk, a, m,
                                             alo, mlo, Tn, cold, j) == 2) {
                a += alo;
                m += mlo;
            }
            af = a;
            mf = m;
            Tc = Tn;
            rest_w = __ballot(act && !rest_bits(af, mf)) == 0;
        }
        if (act) {
            as[local] = a;
            am[local] = m;
            if (beta) beta[local] = flagged ? solid_fraction(T0c) - kXmax - 0.0f : solid_fraction(Tc) - af - mf;
        }
        rest[w] = rest_w ? 1 : 0;
    }
}

__global__ void reset_counters_kernel(unsigned* c) {
    if (threadIdx.x < 2) c[threadIdx.x] = 0u;
}

// records for at most this many waves per launch; more waves than that which
// need the network take the plain steps of those blocks instead
constexpr int64_t kMaxRecords = (int64_t)1 << 16;

hipError_t surrogate_prepare(MlpState& s, int64_t waves, hipStream_t st) {
    const int64_t need = waves < kMaxRecords ? (waves > 0 ? waves : 1) : kMaxRecords;
    if (need > s.rec_cap) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        if (s.recs) (void)hipFree(s.recs);
        s.recs = nullptr;
        s.rec_cap = 0;
        if ((e = hipMalloc(&s.recs, (size_t)need * sizeof(SurrogateRecord))) != hipSuccess) return e;
        s.rec_cap = need;
    }
    if (!s.counters) {
        hipError_t e = hipMalloc((void**)&s.counters, 2 * sizeof(unsigned));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, st, s.counters);
    return hipGetLastError();
}

hipError_t launch_surrogate(const MlpState& s, const PointGeom& pg, int W, const SrcRec* tab, EnvSet env, int Kl,
                            int Ks, float dt, ScanArgs sa, float* beta, float* as, float* am, int64_t li,
                            hipStream_t st) {
    if (pg.count <= 0) return hipSuccess;
    SurrogateRecord* recs = static_cast<SurrogateRecord*>(s.recs);
    unsigned* cur = s.counters + (li & 1);
    unsigned* nxt = s.counters + ((li + 1) & 1);
    const int64_t cap = s.rec_cap;
    const MlpNorm& nrm = s.norm;
    const dim3 grid((unsigned)((pg.count + kFusedBlock - 1) / kFusedBlock)), block(kFusedBlock);
    switch (W) {
        case 1: hipLaunchKernelGGL(fused_surrogate_kernel<1>, grid, block, 0, st, pg, tab, env, Kl, Ks, dt, sa, nrm, beta, as, am, recs, cur, cap); break;
        case 2: hipLaunchKernelGGL(fused_surrogate_kernel<2>, grid, block, 0, st, pg, tab, env, Kl, Ks, dt, sa, nrm, beta, as, am, recs, cur, cap); break;
        case 3: hipLaunchKernelGGL(fused_surrogate_kernel<3>, grid, block, 0, st, pg, tab, env, Kl, Ks, dt, sa, nrm, beta, as, am, recs, cur, cap); break;
        case 4: hipLaunchKernelGGL(fused_surrogate_kernel<4>, grid, block, 0, st, pg, tab, env, Kl, Ks, dt, sa, nrm, beta, as, am, recs, cur, cap); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 rg(256), rb(256);
    switch (W) {
        case 1: hipLaunchKernelGGL(surrogate_resume_kernel<1>, rg, rb, 0, st, pg, tab, env, Kl, Ks, dt, sa, nrm, beta, as, am, recs, cur, nxt, cap, s.frag); break;
        case 2: hipLaunchKernelGGL(surrogate_resume_kernel<2>, rg, rb, 0, st, pg, tab, env, Kl, Ks, dt, sa, nrm, beta, as, am, recs, cur, nxt, cap, s.frag); break;
        case 3: hipLaunchKernelGGL(surrogate_resume_kernel<3>, rg, rb, 0, st, pg, tab, env, Kl, Ks, dt, sa, nrm, beta, as, am, recs, cur, nxt, cap, s.frag); break;
        case 4: hipLaunchKernelGGL(surrogate_resume_kernel<4>, rg, rb, 0, st, pg, tab, env, Kl, Ks, dt, sa, nrm, beta, as, am, recs, cur, nxt, cap, s.frag); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// the correction g at a given temperature, in place (training targets)
__global__ __launch_bounds__(256) void correct_kernel(const float* __restrict__ T, float* __restrict__ beta,
                                                     float* __restrict__ as, float* __restrict__ am, int64_t n,
                                                     bool assign) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float a = as[i], m = am[i];
    const float Ti = T[i];
    beta[i] = correct(Ti, alpha_eq(Ti), a, m, assign);
    as[i] = a;
    am[i] = m;
}

hipError_t launch_correct(const float* T, float* beta, float* as, float* am, int64_t n, bool assign, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(correct_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, T, beta, as, am, n,
                       assign);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
hipError_t mlp_alloc(MlpState& s) {
    if (s.master) return hipSuccess;
    hipError_t e;
    if ((e = hipMalloc((void**)&s.master, kMlpParams * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&s.adam_m, kMlpParams * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&s.adam_v, kMlpParams * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&s.grad, kMlpParams * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&s.loss, sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&s.frag, kFragTotal * sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&s.partial, (size_t)kMaxTrainWaves * (kMlpParams + 1) * sizeof(float))) != hipSuccess)
        return e;
    s.partial_waves = kMaxTrainWaves;
    return hipSuccess;
}

void mlp_free(MlpState& s) {
    for (void* p : {(void*)s.master, (void*)s.adam_m, (void*)s.adam_v, (void*)s.grad, (void*)s.loss, (void*)s.frag,
                    (void*)s.partial, (void*)s.recs, (void*)s.counters})
        if (p) (void)hipFree(p);
    s = MlpState{};
}


hipError_t launch_surrogate_call(const MlpState& s, const PointGeom& pg, int W, const SrcRec* tab, const EnvRec* env,
                                 const int32_t* env_fc, const uint8_t* below, uint8_t* rest, int64_t n_waves,
                                 int64_t l0, int64_t nl, int Kl, int Ks, int64_t n_steps, float dt, ScanArgs sa,
                                 float* beta, float* as, float* am, uint32_t* cand, unsigned* counts,
                                 unsigned long long* stats, hipStream_t st) {
    if (n_waves <= 0 || nl <= 0) return hipSuccess;
    hipError_t e = launch_chunk_list(pg, below, rest, n_waves, l0, nl, fminf(sa.T0, sa.Tclamp), beta, as, am, cand,
                                     counts, stats, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, st, s.counters);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    SurrogateRecord* recs = static_cast<SurrogateRecord*>(s.recs);
    const int64_t cap = s.rec_cap;
    const MlpNorm& nrm = s.norm;
    const dim3 grid = call_grid(n_waves), block(kCallBlock), rg(256), rb(256);
    switch (W) {
#define MSTRUCT_SURROGATE_CALL(WW)                                                                                   \
    case WW:                                                                                                         \
        hipLaunchKernelGGL(fused_surrogate_call_kernel<WW>, grid, block, 0, st, pg, tab, env, env_fc, below, rest,    \
                           n_waves, l0, nl, Kl, Ks, n_steps, dt, sa, nrm, beta, as, am, cand, counts, counts + 1,     \
                           stats, recs, s.counters, cap);                                                            \
        if ((e = hipGetLastError()) != hipSuccess) return e;                                                         \
        hipLaunchKernelGGL(surrogate_resume_call_kernel<WW>, rg, rb, 0, st, pg, tab, env, env_fc, below, rest,        \
                           n_waves, l0, nl, Kl, Ks, n_steps, dt, sa, nrm, beta, as, am, recs, s.counters, cap,        \
                           s.frag, stats);                                                                           \
        break;
        MSTRUCT_SURROGATE_CALL(1)
        MSTRUCT_SURROGATE_CALL(2)
        MSTRUCT_SURROGATE_CALL(3)
        MSTRUCT_SURROGATE_CALL(4)
#undef MSTRUCT_SURROGATE_CALL
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mstruct
