// The first encoder layer E1 (Table I's encoder, first 3x3 stride-2
// convolution + leaky ReLU) read straight from the coarse maps: its input x0
// has two channels (f d / 256 and I / 256), so a direct stencil -- each thread
// one output pixel and eight output channels, 18 fused multiply-adds per
// channel -- does in a few registers what an implicit GEMM would pad to a full
// channel chunk.  The weights are widened to FP32 in LDS once per workgroup
// and read as one broadcast per wave (a wave owns one group of eight output
// channels); the x0 patch of the tile is built in LDS as FP32.  The LDS is
// sized by the layer's width, so narrow layers keep many workgroups per CU.
//
// INT8 networks run the same stencil on the quantised layer's codes: x0
// quantised with the input scale (127 / amax of x0, as the convolution's
// staging does), the weights' INT8 codes, and the products summed in FP32,
// which is exact here (at most 18 x 127 x 127 < 2^24, every partial sum an
// integer), so the sum equals the matrix units' INT32 sum; then the same
// dequantisation (sum x s_in s_w), bias, leaky ReLU, BF16 store and record
// of the output's max |value| as the convolution's epilogue.
#include <algorithm>
#include "kernels.h"

namespace sv {

constexpr int E1_TW = 16, E1_TH = 4;                      // output tile
constexpr int E1_PW = 2 * E1_TW + 1, E1_PH = 2 * E1_TH + 1;  // x0 patch (stride 2, pad 1)
constexpr int E1_MAXC = 256;
constexpr int E1_XN = (2 * E1_PH * E1_PW + 3) & ~3;        // x0 patch floats, 16-byte multiple

// Dynamic LDS: x[2][E1_PH * E1_PW] (padded to E1_XN floats), then
// w[9 * 2][c1] ([tap * 2 + channel][output channel]), bias[c1] and, for INT8,
// the dequantisation factors scale[c1] = s_in * s_w.
struct Enc1Smem {
    float *x[2];
    float *w;
    float *bias;
    float *scale;
    int c1;
};
static inline size_t enc1_lds_bytes(int c1) { return sizeof(float) * ((size_t)E1_XN + 20 * (size_t)c1); }

__device__ __forceinline__ Enc1Smem enc1_smem(float *dyn, int c1) {
    Enc1Smem sm;
    sm.x[0] = dyn;
    sm.x[1] = dyn + E1_PH * E1_PW;
    sm.w = dyn + E1_XN;
    sm.bias = sm.w + 18 * c1;
    sm.scale = sm.bias + c1;
    sm.c1 = c1;
    return sm;
}

template <int DT>
__device__ __forceinline__ void enc1_weights(const Enc1Smem &sm, const typename Elem<DT>::T *__restrict__ wpk,
                                             int n_pad, int cin_pad, const float *__restrict__ bias, int c1) {
    for (int e = threadIdx.x; e < 18 * c1; e += 256) {
        const int tc = e / c1, n = e - tc * c1;
        const int tap = tc >> 1, c = tc & 1;
        sm.w[tc * c1 + n] = Elem<DT>::load(wpk + ((size_t)tap * n_pad + n) * cin_pad + c);
    }
    for (int n = threadIdx.x; n < c1; n += 256) sm.bias[n] = bias[n];
}

// stored element type of E1's output (INT8 layers store BF16 maps)
template <int DT> using E1Out = typename Elem<DT == SV_I8 ? SV_BF16 : DT>::T;

// INT8 pass state: the input's quantisation step and scale, the weights'
// per-channel scales, and this workgroup's running max |stored value|
struct Enc1Q {
    float qinv, s_in;
    const float *wscale;
    float lmax;
};

// The raw coarse bytes of one tile's x0 patch, entries tid and tid + 256 of
// the E1_PH x E1_PW patch per thread: loaded ahead of their use (before the
// weights, and during the previous tile's arithmetic), converted when they
// are written to LDS.  Entries outside the map read byte 0 and are zeroed.
static_assert(E1_PH * E1_PW <= 512, "two patch entries per thread");
struct E1Patch {
    uint32_t d[2], im[2];
    bool in[2];
};

__device__ __forceinline__ void enc1_fetch(E1Patch &P, const uint8_t *__restrict__ disp,
                                           const uint8_t *__restrict__ img, int h0, int w0, int oy0, int ox0) {
    const int iy0 = 2 * oy0 - 1, ix0 = 2 * ox0 - 1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int e = threadIdx.x + 256 * k;
        const int py = e / E1_PW, px = e - py * E1_PW;
        const int y = iy0 + py, x = ix0 + px;
        P.in[k] = e < E1_PH * E1_PW && y >= 0 && y < h0 && x >= 0 && x < w0;
        const size_t o = P.in[k] ? (size_t)y * w0 + x : 0;
        P.d[k] = disp[o];
        P.im[k] = img[o];
    }
}

template <int DT>
__device__ __forceinline__ void enc1_put(const E1Patch &P, const Enc1Smem &sm, float scale0, const Enc1Q &q) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int e = threadIdx.x + 256 * k;
        if (e >= E1_PH * E1_PW) continue;
        float a = 0.f, c = 0.f;
        if (P.in[k]) {
            a = scale0 * (float)P.d[k];
            c = (float)P.im[k] * (1.0f / 256.0f);
            if constexpr (DT == SV_I8) {  // the INT8 codes, as values
                a = fminf(fmaxf(rintf(a * q.qinv), -127.0f), 127.0f);
                c = fminf(fmaxf(rintf(c * q.qinv), -127.0f), 127.0f);
            }
        }
        sm.x[0][e] = a;
        sm.x[1][e] = c;
    }
}

// One tile's arithmetic and stores, the patch already in LDS (a barrier
// after enc1_put): output rows [oy0, oy0 + E1_TH) and columns
// [ox0, ox0 + E1_TW) of an h1 x w1 map.  Ends with a barrier, after which
// the patch can take the next tile.
template <int DT>
__device__ __forceinline__ void enc1_compute(const Enc1Smem &sm, int h1, int w1, int c1, int oy0, int ox0,
                                             E1Out<DT> *__restrict__ out, Enc1Q &q) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int grp = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform channel group
    const int tx = lane & (E1_TW - 1), ty = lane / E1_TW;
    const int oy = oy0 + ty, ox = ox0 + tx;
    if (oy < h1 && ox < w1) {
        // the 18 input values of this pixel, tap-major, disparity channel first
        float xin[18];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int u = t / 3, v = t % 3;
            const int q = (2 * ty + u) * E1_PW + 2 * tx + v;
            xin[2 * t] = sm.x[0][q];
            xin[2 * t + 1] = sm.x[1][q];
        }
        for (int g = grp; g * 8 < c1; g += 4) {
            const int n0 = g * 8;
            float acc[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] = 0.f;
#pragma unroll
            for (int k = 0; k < 18; ++k) {
                const f32x4 wa = *(const f32x4 *)&sm.w[k * c1 + n0];
                const f32x4 wb = *(const f32x4 *)&sm.w[k * c1 + n0 + 4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    acc[i] = fmaf(wa[i], xin[k], acc[i]);
                    acc[4 + i] = fmaf(wb[i], xin[k], acc[4 + i]);
                }
            }
            float r[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                float a = acc[i];
                if constexpr (DT == SV_I8) a = acc[i] * sm.scale[n0 + i];
                const float s = a + sm.bias[n0 + i];
                r[i] = s > 0.f ? s : 0.1f * s;
            }
            E1Out<DT> *op = out + ((size_t)oy * w1 + ox) * c1 + n0;
            if constexpr (DT == SV_I8) {
                u16x8 v;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    v[i] = Elem<SV_BF16>::make(r[i]);
                    q.lmax = fmaxf(q.lmax, fabsf(bf16_bits_to_f32(v[i])));
                }
                *(u16x8 *)op = v;
            } else if constexpr (DT == SV_F32) {
                *(f32x4 *)op = f32x4{r[0], r[1], r[2], r[3]};
                *(f32x4 *)(op + 4) = f32x4{r[4], r[5], r[6], r[7]};
            } else {
                u16x8 q;
#pragma unroll
                for (int i = 0; i < 8; ++i) q[i] = Elem<DT>::make(r[i]);
                *(u16x8 *)op = q;
            }
        }
    }
    __syncthreads();  // the patch is reused by the next tile of a persistent loop
}

// Uniform batch: a persistent grid walks the tiles (image-major), so the
// weights are widened into LDS once per workgroup.
template <int DT>
__global__ void __launch_bounds__(256)
k_enc1(const uint8_t *__restrict__ disp, const uint8_t *__restrict__ img, float scale0, int B, int h0, int w0,
       int h1, int w1, int c1, const typename Elem<DT>::T *__restrict__ wpk, int n_pad, int cin_pad,
       const float *__restrict__ bias, E1Out<DT> *__restrict__ out, const float *__restrict__ wscale,
       const uint32_t *__restrict__ amax_in, uint32_t *__restrict__ amax_out) {
    extern __shared__ __attribute__((aligned(16))) float e1_dyn[];
    const Enc1Smem sm = enc1_smem(e1_dyn, c1);
    const int tx = cdiv_d(w1, E1_TW), ty = cdiv_d(h1, E1_TH);
    const int per = tx * ty, total = per * B;
    // the first tile's patch loads go out before the weights'
    E1Patch P;
    if ((int)blockIdx.x < total) {
        const int b = blockIdx.x / per, r = blockIdx.x - b * per;
        const size_t i0 = (size_t)b * h0 * w0;
        enc1_fetch(P, disp + i0, img + i0, h0, w0, (r / tx) * E1_TH, (r % tx) * E1_TW);
    }
    enc1_weights<DT>(sm, wpk, n_pad, cin_pad, bias, c1);
    Enc1Q q{0.f, 0.f, wscale, 0.f};
    if constexpr (DT == SV_I8) {
        // the input scale from x0's recorded maxima (lane j reads word j)
        float m = __uint_as_float(amax_in[threadIdx.x & (AMAX_SUB - 1)]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        q.qinv = m > 0.f ? 127.0f / m : 0.f;
        q.s_in = m / 127.0f;
        for (int n = threadIdx.x; n < c1; n += 256) sm.scale[n] = q.s_in * wscale[n];
    }
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int b = t / per, r = t - b * per;
        const size_t o1 = (size_t)b * h1 * w1;
        enc1_put<DT>(P, sm, scale0, q);
        __syncthreads();
        const int tn = t + (int)gridDim.x;  // the next tile's patch, loaded during this one's arithmetic
        if (tn < total) {
            const int bn = tn / per, rn = tn - bn * per;
            const size_t in0 = (size_t)bn * h0 * w0;
            enc1_fetch(P, disp + in0, img + in0, h0, w0, (rn / tx) * E1_TH, (rn % tx) * E1_TW);
        }
        enc1_compute<DT>(sm, h1, w1, c1, (r / tx) * E1_TH, (r % tx) * E1_TW, out + o1 * c1, q);
    }
    if constexpr (DT == SV_I8) {
        // the workgroup's max: waves through the (free) patch area, then one
        // atomic per workgroup
        float m = q.lmax;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if ((threadIdx.x & 63) == 0) sm.x[0][threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            const float w = fmaxf(fmaxf(sm.x[0][0], sm.x[0][1]), fmaxf(sm.x[0][2], sm.x[0][3]));
            atomicMax(amax_out + (blockIdx.x & (AMAX_SUB - 1)), __float_as_uint(w));
        }
    }
}

// Persistent variant over the pair table (flattened per-level buffers).
template <int DT>
__global__ void __launch_bounds__(256)
k_enc1_tab(const PairTable *__restrict__ tab, const uint8_t *__restrict__ disp, const uint8_t *__restrict__ img,
           float scale0, int c1, const typename Elem<DT>::T *__restrict__ wpk, int n_pad, int cin_pad,
           const float *__restrict__ bias, typename Elem<DT>::T *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) float e1_dyn[];
    const Enc1Smem sm = enc1_smem(e1_dyn, c1);
    enc1_weights<DT>(sm, wpk, n_pad, cin_pad, bias, c1);
    const int n = tab->n;
    const int *cum = tab->cum[BS_E1];
    const int total = cum[n];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = table_find(cum, n, t);
        const PairGeo &g = tab->pair[i];
        const int local = t - cum[i];
        const int tx = cdiv_d(g.w[1], E1_TW);
        Enc1Q q{0.f, 0.f, nullptr, 0.f};  // (no INT8 pair-table path)
        E1Patch P;
        enc1_fetch(P, disp + g.off[0], img + g.off[0], g.h[0], g.w[0], (local / tx) * E1_TH, (local % tx) * E1_TW);
        enc1_put<DT>(P, sm, scale0, q);
        __syncthreads();
        enc1_compute<DT>(sm, g.h[1], g.w[1], c1, (local / tx) * E1_TH, (local % tx) * E1_TW,
                         out + (size_t)g.off[1] * c1, q);
    }
}

int enc1_tiles(int h1, int w1) { return cdiv(h1, E1_TH) * cdiv(w1, E1_TW); }

sv_status launch_enc1(int dtype, const uint8_t *disp, const uint8_t *img, float scale0, int B, int h0, int w0,
                      int h1, int w1, int c1, const void *wpk, int n_pad, int cin_pad, const float *bias,
                      void *out, hipStream_t st, const float *wscale, const uint32_t *amax_in,
                      uint32_t *amax_out) {
    if (c1 < 8 || c1 > E1_MAXC || c1 % 8) return SV_ERR_UNSUPPORTED;
    if (dtype == SV_I8 && (!wscale || !amax_in || !amax_out)) return SV_ERR_NULL;
    const long long tiles = (long long)enc1_tiles(h1, w1) * B;
    if (tiles >= (1ll << 31)) return SV_ERR_SHAPE;
    switch (dtype) {
#define SV_E1(D, TW, TO)                                                                                \
    case D: {                                                                                           \
        const dim3 grid((unsigned)resident_grid((const void *)k_enc1<D>, enc1_lds_bytes(c1), tiles));     \
        hipLaunchKernelGGL(k_enc1<D>, grid, dim3(256), enc1_lds_bytes(c1), st, disp, img, scale0, B, h0, \
                           w0, h1, w1, c1, (const TW *)wpk, n_pad, cin_pad, bias, (TO *)out, wscale,    \
                           amax_in, amax_out);                                                          \
        break;                                                                                          \
    }
        SV_E1(SV_F32, float, float)
        SV_E1(SV_BF16, uint16_t, uint16_t)
        SV_E1(SV_F16, uint16_t, uint16_t)
        SV_E1(SV_I8, int8_t, uint16_t)
#undef SV_E1
    default: return SV_ERR_DTYPE;
    }
    SV_LAUNCH_CHECK("k_enc1");
    return SV_OK;
}

sv_status launch_enc1_tab(int dtype, const PairTable *tab, int grid, const uint8_t *disp, const uint8_t *img,
                          float scale0, int c1, const void *wpk, int n_pad, int cin_pad, const float *bias,
                          void *out, hipStream_t st) {
    if (c1 < 8 || c1 > E1_MAXC || c1 % 8) return SV_ERR_UNSUPPORTED;
    switch (dtype) {
#define SV_E1T(D, T)                                                                                    \
    case D:                                                                                             \
        hipLaunchKernelGGL(k_enc1_tab<D>, dim3(resident_grid((const void *)k_enc1_tab<D>, enc1_lds_bytes(c1), grid)), \
                           dim3(256), enc1_lds_bytes(c1), st, tab, disp, img,                           \
                           scale0, c1,                                                                  \
                           (const T *)wpk, n_pad, cin_pad, bias, (T *)out);                             \
        break;
        SV_E1T(SV_F32, float)
        SV_E1T(SV_BF16, uint16_t)
        SV_E1T(SV_F16, uint16_t)
#undef SV_E1T
    default: return SV_ERR_DTYPE;
    }
    SV_LAUNCH_CHECK("k_enc1_tab");
    return SV_OK;
}

}  // namespace sv
