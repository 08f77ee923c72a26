// The matrix-unit steps the convolutions use (forward, backward and the
// fused latent kernel): one 16 x 16 output block, k values per lane per step
// (GS), operands as LDS vectors of the compute dtype.
#pragma once

#include "kernels.h"

namespace sv {

template <int DT> struct Mfma;

template <> struct Mfma<SV_BF16> {
    static constexpr int GS = 8;  // k values per lane per step
    typedef uint16_t T;
    typedef u16x8 vec;
    typedef f32x4 acc;
    static __device__ __forceinline__ f32x4 run(vec a, vec b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
};

template <> struct Mfma<SV_F16> {
    static constexpr int GS = 8;
    typedef uint16_t T;
    typedef u16x8 vec;
    typedef f32x4 acc;
    static __device__ __forceinline__ f32x4 run(vec a, vec b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
};

// FP32: four 16x16x4 steps; lane group g supplies k = 4g + i to step i for
// both operands, so A and B agree on the k order.
template <> struct Mfma<SV_F32> {
    static constexpr int GS = 4;
    typedef float T;
    typedef f32x4 vec;
    typedef f32x4 acc;
    static __device__ __forceinline__ f32x4 run(vec a, vec b, f32x4 c) {
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
        return c;
    }
};

// INT8: eight codes per lane per step, exact INT32 sums.
template <> struct Mfma<SV_I8> {
    static constexpr int GS = 8;
    typedef int8_t T;
    typedef i8x8 vec;
    typedef i32x4 acc;
    static __device__ __forceinline__ i32x4 run(vec a, vec b, i32x4 c) {
        return __builtin_amdgcn_mfma_i32_16x16x32_i8(__builtin_bit_cast(long, a), __builtin_bit_cast(long, b), c,
                                                     0, 0, 0);
    }
};

}  // namespace sv
