// Internal helpers shared by the HIP sources of libsv.so (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/sv.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef int8_t i8x8 __attribute__((ext_vector_type(8)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

namespace sv {

// Records the HIP error text for sv_last_error() and maps it to SV_ERR_HIP.
sv_status hip_fail(hipError_t e, const char *where);

#define SV_HIP(call)                                                 \
    do {                                                             \
        hipError_t e_ = (call);                                      \
        if (e_ != hipSuccess) return ::sv::hip_fail(e_, #call);      \
    } while (0)

#define SV_LAUNCH_CHECK(name)                                        \
    do {                                                             \
        hipError_t e_ = hipGetLastError();                           \
        if (e_ != hipSuccess) return ::sv::hip_fail(e_, name);       \
    } while (0)

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }
__device__ __forceinline__ int cdiv_d(int a, int b) { return (a + b - 1) / b; }
static inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ---- storage types of the network's activations and weights ------------------
// FP32 -> BF16 / FP16 with round-to-nearest-even.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    return __builtin_bit_cast(uint16_t, (__bf16)f);  // v_cvt_pk_bf16_f32, round to nearest even
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f32_to_f16_bits(float f) {
    _Float16 h = (_Float16)f;  // IEEE round-to-nearest-even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_bits_to_f32(uint16_t h) {
    return (float)__builtin_bit_cast(_Float16, h);
}

// Element traits: how a stored value converts to and from FP32.
template <int DT> struct Elem;
template <> struct Elem<SV_F32> {
    typedef float T;
    static __device__ __forceinline__ float load(const T *p) { return *p; }
    static __device__ __forceinline__ T make(float f) { return f; }
};
template <> struct Elem<SV_BF16> {
    typedef uint16_t T;
    static __device__ __forceinline__ float load(const T *p) { return bf16_bits_to_f32(*p); }
    static __device__ __forceinline__ T make(float f) { return f32_to_bf16_bits(f); }
};
template <> struct Elem<SV_F16> {
    typedef uint16_t T;
    static __device__ __forceinline__ float load(const T *p) { return f16_bits_to_f32(*p); }
    static __device__ __forceinline__ T make(float f) { return f32_to_f16_bits(f); }
};

// bytes of a stored activation (INT8 layers store BF16)
// INT8 codes (clamped to +-127, round to nearest even)
template <> struct Elem<SV_I8> {
    typedef int8_t T;
    static __device__ __forceinline__ float load(const T *p) { return (float)*p; }
    static __device__ __forceinline__ T make(float f) {
        return (int8_t)(int)fminf(fmaxf(rintf(f), -127.0f), 127.0f);
    }
};

static inline int dtype_bytes(int dt) { return dt == SV_F32 ? 4 : 2; }

// Bilinear source index pair and weight along one axis for output index o of a
// resize from n_in to n_out samples with half-pixel centres (no corner
// alignment): s = (o + 1/2) n_in / n_out - 1/2 clamped at 0.  The position is
// formed as the exact rational ((2o+1) n_in - n_out) / (2 n_out), so i0 is an
// integer quotient and only the weight is rounded (once).
__device__ __forceinline__ void bilin(int o, int n_in, int n_out, int &i0, int &i1, float &lam) {
    const int num = (2 * o + 1) * n_in - n_out;
    if (num <= 0) {
        i0 = 0;
        lam = 0.0f;
    } else {
        const int den = 2 * n_out;
        i0 = num / den;
        lam = (float)(num - i0 * den) / (float)den;
    }
    i1 = min(i0 + 1, n_in - 1);
}

}  // namespace sv
