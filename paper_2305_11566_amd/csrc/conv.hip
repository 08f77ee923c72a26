// Convolutions of the refinement network (Table I) as implicit GEMM on MFMA.
//
// GEMM view: rows = output channels n, columns = output pixels m, reduction
// over k = (tap, input channel).  The MFMA A operand is a 16 x k slice of the
// weights and B a k x 16 slice of the input, so each lane of the 16x16
// result holds four consecutive output channels of one pixel, which the
// epilogue stores as one NHWC vector.
//
// A workgroup (4 waves) owns an output tile of TH rows x 16 columns of one
// image and TN output channels.  For each chunk of KC input channels it
// stages into LDS
//   * the input patch (tile plus halo), gathered from up to two sources:
//     a same-level NHWC map, a map bilinearly resized on the fly from a
//     coarser level (the decoder's upsampling), or the network input x0 built
//     from the uint8 coarse disparity and reduced left image; out-of-image
//     pixels and channels past Cin are zeros (the zero padding);
//   * the chunk of packed weights for all taps and the tile's TN channels.
// The reduction then runs over (tap, channel group) pairs straight out of
// LDS: lane group g (lanes 16g..16g+15) takes pair 4*step + g, so a step
// covers four pairs whatever the tap count, and Cin = 2 (the first layer)
// wastes little.  Accumulation is FP32 for every storage type.  The order of
// the reduction is fixed by the base chunk and the step, not by the tile
// shape, so every tile shape gives bitwise-identical results.  The kernel
// templates live in conv_impl.h and are instantiated per compute dtype in
// conv_f32.hip / conv_bf16.hip / conv_f16.hip; this file holds the tile
// table, the dispatch and the weight packing.
#include <algorithm>
#include <cstdio>
#include <mutex>

#include "conv_impl.h"

namespace sv {

// ---- tile configurations ---------------------------------------------------------
// A configuration id is a tile shape plus a reduction split:
// id = tile + kNumTiles * (ksplit - 1), ksplit = 1 .. kMaxSplit.  A split only
// applies to uniform launches that bring a partial-sum buffer.
struct CfgDesc { int TH, TN, WM, KCM; const char *name; };
static const CfgDesc kCfgs[] = {
#define SV_CFG(i, TH, TN, WM, KCM, name) {TH, TN, WM, KCM, name},
    SV_CONV_CFGS(SV_CFG)
#undef SV_CFG
};
static constexpr int kNumTiles = (int)(sizeof(kCfgs) / sizeof(kCfgs[0]));
static constexpr int kMaxSplit = CONV_MAX_SPLIT;
static constexpr int kFallbackTile = 5;  // th4_tn16
int conv_num_tiles() { return kNumTiles; }
int conv_num_cfgs() { return kNumTiles * kMaxSplit; }

const char *conv_cfg_name(int cfg) {
    static char names[kNumTiles * kMaxSplit][32];
    static std::once_flag once;
    std::call_once(once, [] {
        for (int i = 0; i < kNumTiles * kMaxSplit; ++i) {
            const int t = i % kNumTiles, sp = i / kNumTiles + 1;
            if (sp == 1) snprintf(names[i], sizeof names[i], "%s", kCfgs[t].name);
            else snprintf(names[i], sizeof names[i], "%s_s%d", kCfgs[t].name, sp);
        }
    });
    return (cfg >= 0 && cfg < conv_num_cfgs()) ? names[cfg] : "?";
}

sv_status launch_conv_f32(int ks, int stride, int cfg, const ConvParams &p, int pg, hipStream_t st);
sv_status launch_split_sum_f32(const ConvParams &p, hipStream_t st);
sv_status launch_split_sum_bf16(const ConvParams &p, hipStream_t st);
sv_status launch_split_sum_f16(const ConvParams &p, hipStream_t st);
sv_status launch_conv_bf16(int ks, int stride, int cfg, const ConvParams &p, int pg, hipStream_t st);
sv_status launch_conv_f16(int ks, int stride, int cfg, const ConvParams &p, int pg, hipStream_t st);
bool conv_fits_f32(int ks, int stride, int tile);
bool conv_fits_bf16(int ks, int stride, int tile);
bool conv_fits_f16(int ks, int stride, int tile);
sv_status launch_conv_i8(int ks, int stride, int cfg, const ConvParams &p, int pg, hipStream_t st);
bool conv_fits_i8(int ks, int stride, int tile);
#define SV_CONV5_DECL(S, dt)                                                                      \
    sv_status launch_conv5_s##S##_##dt(int cfg, const ConvParams &p, int pg, hipStream_t st); \
    bool conv5_fits_s##S##_##dt(int tile);
SV_CONV5_DECL(1, f32) SV_CONV5_DECL(2, f32) SV_CONV5_DECL(1, bf16) SV_CONV5_DECL(2, bf16)
SV_CONV5_DECL(1, f16) SV_CONV5_DECL(2, f16)
#undef SV_CONV5_DECL

static bool fits_any(int dtype, int ks, int stride, int tile) {
    if (ks == 5) {
        if (stride != 1 && stride != 2) return false;
        switch (dtype) {
        case SV_F32: return stride == 1 ? conv5_fits_s1_f32(tile) : conv5_fits_s2_f32(tile);
        case SV_BF16: return stride == 1 ? conv5_fits_s1_bf16(tile) : conv5_fits_s2_bf16(tile);
        case SV_F16: return stride == 1 ? conv5_fits_s1_f16(tile) : conv5_fits_s2_f16(tile);
        default: return false;
        }
    }
    switch (dtype) {
    case SV_F32: return conv_fits_f32(ks, stride, tile);
    case SV_BF16: return conv_fits_bf16(ks, stride, tile);
    case SV_F16: return conv_fits_f16(ks, stride, tile);
    case SV_I8: return conv_fits_i8(ks, stride, tile);
    default: return false;
    }
}

// A configuration whose tile shape does not fit the LDS for this kernel size
// and stride runs as th4_tn16 (which fits every case) with the same split;
// the tile shape does not change results.
int conv_resolve_cfg(int dtype, int ks, int stride, int cfg) {
    if (cfg < 0 || cfg >= conv_num_cfgs()) return cfg;
    if (dtype != SV_F32 && dtype != SV_BF16 && dtype != SV_F16 && dtype != SV_I8) return cfg;
    const int tile = cfg % kNumTiles;
    return fits_any(dtype, ks, stride, tile) ? cfg : cfg - tile + kFallbackTile;
}

static sv_status launch_any(int dtype, int ks, int stride, int tile, const ConvParams &p, int pg,
                            hipStream_t st) {
    if (ks == 5) {
        if (stride != 1 && stride != 2) return SV_ERR_UNSUPPORTED;
        switch (dtype) {
        case SV_F32:
            return stride == 1 ? launch_conv5_s1_f32(tile, p, pg, st) : launch_conv5_s2_f32(tile, p, pg, st);
        case SV_BF16:
            return stride == 1 ? launch_conv5_s1_bf16(tile, p, pg, st) : launch_conv5_s2_bf16(tile, p, pg, st);
        case SV_F16:
            return stride == 1 ? launch_conv5_s1_f16(tile, p, pg, st) : launch_conv5_s2_f16(tile, p, pg, st);
        default: return SV_ERR_DTYPE;
        }
    }
    switch (dtype) {
    case SV_F32: return launch_conv_f32(ks, stride, tile, p, pg, st);
    case SV_BF16: return launch_conv_bf16(ks, stride, tile, p, pg, st);
    case SV_F16: return launch_conv_f16(ks, stride, tile, p, pg, st);
    case SV_I8:
        if (ks == 5) return SV_ERR_UNSUPPORTED;
        return launch_conv_i8(ks, stride, tile, p, pg, st);
    default: return SV_ERR_DTYPE;
    }
}

int conv_effective_split(int dtype, int cfg, int Cin, long long npix, int n_pad, const float *part,
                         size_t part_bytes) {
    if (dtype == SV_I8) return 1;  // integer sums are kept whole
    int ksplit = cfg / kNumTiles + 1;
    // at most one split per base chunk of input channels, and only when the
    // partial sums fit the caller's buffer; otherwise one pass
    const int kcb = dtype == SV_F32 ? 16 : 32;
    ksplit = std::min(ksplit, cdiv(Cin, kcb));
    const size_t need = (size_t)ksplit * (size_t)npix * n_pad * sizeof(float);
    if (!part || need > part_bytes) ksplit = 1;
    return ksplit;
}

sv_status launch_conv_split(int dtype, int ks, int stride, int cfg, const ConvParams &p0, hipStream_t st,
                            int *ksplit_used) {
    if (cfg < 0 || cfg >= conv_num_cfgs()) return SV_ERR_RANGE;
    cfg = conv_resolve_cfg(dtype, ks, stride, cfg);
    ConvParams p = p0;
    p.ksplit = conv_effective_split(dtype, cfg, p.Cin, (long long)p.B * p.Ho * p.Wo, p.n_pad, p.part,
                                    p.part_bytes);
    if (p.ophase) p.ksplit = 1;  // a phase launch writes its pixels straight into the full map
    if (p.proj_out) {
        // the projection epilogue needs whole sums and every channel in each wave
        if (!conv_cfg_projects(cfg % kNumTiles, p.Cout)) return SV_ERR_UNSUPPORTED;
        p.ksplit = 1;
    }
    if (ksplit_used) *ksplit_used = p.ksplit > 1 ? p.ksplit : 1;
    return launch_any(dtype, ks, stride, cfg % kNumTiles, p, 0, st);
}

sv_status launch_split_sum(int dtype, const ConvParams &p0, int ksplit, hipStream_t st) {
    if (ksplit <= 1) return SV_OK;
    ConvParams p = p0;
    p.ksplit = ksplit;
    p.defer_sum = 0;
    switch (dtype) {
    case SV_F32: return launch_split_sum_f32(p, st);
    case SV_BF16: return launch_split_sum_bf16(p, st);
    case SV_F16: return launch_split_sum_f16(p, st);
    default: return SV_ERR_DTYPE;  // INT8 never splits
    }
}

sv_status launch_conv(int dtype, int ks, int stride, int cfg, const ConvParams &p0, hipStream_t st) {
    return launch_conv_split(dtype, ks, stride, cfg, p0, st, nullptr);
}

sv_status launch_conv_tab(int dtype, int ks, int stride, int cfg, const ConvParams &p0, int grid,
                          hipStream_t st) {
    if (!p0.tab || grid <= 0) return SV_ERR_RANGE;
    if (cfg < 0 || cfg >= conv_num_cfgs()) return SV_ERR_RANGE;
    cfg = conv_resolve_cfg(dtype, ks, stride, cfg);
    if (p0.proj_out && !conv_cfg_projects(cfg % kNumTiles, p0.Cout))
        return SV_ERR_UNSUPPORTED;
    ConvParams p = p0;
    p.ksplit = 1;  // the persistent path never splits
    return launch_any(dtype, ks, stride, cfg % kNumTiles, p, grid, st);
}

// The tile shape a persistent pair-table launch uses for configuration cfg:
// 16-row tiles (tuned on uniform batches) become the 8-row tile of the same
// width, which runs faster there (twice the resident workgroups and twice
// the tiles to balance over uneven pairs).
int conv_persistent_cfg(int cfg) {
    if (cfg < 0 || cfg >= conv_num_cfgs()) return cfg;
    const CfgDesc &c = kCfgs[cfg % kNumTiles];
    if (c.TH != 16) return cfg;
    for (int t = 0; t < kNumTiles; ++t)
        if (kCfgs[t].TH == 8 && kCfgs[t].TN == c.TN && kCfgs[t].WM == c.WM && kCfgs[t].KCM == c.KCM)
            return t + (cfg / kNumTiles) * kNumTiles;
    return cfg;
}

bool conv_cfg_projects(int cfg, int cout) {
    if (cfg < 0) return false;
    const CfgDesc &c = kCfgs[cfg % kNumTiles];
    return c.TN >= cout && c.WM == 4;  // one channel tile; WN = 4 / WM = 1
}

void conv_cfg_tile(int cfg, int &TH, int &TN) {
    if (cfg < 0 || cfg >= conv_num_cfgs()) cfg = 0;
    TH = kCfgs[cfg % kNumTiles].TH;
    TN = kCfgs[cfg % kNumTiles].TN;
}

// ---- weight packing ---------------------------------------------------------------
// mode 0: forward [tap][n = out][c = in]; mode 1: the final layer, one row
// per source tap; mode 2: adjoint [tap'][n = in][c = out] with the kernel
// flipped (tap' = (k-1-u)*k + (k-1-v)), so the input gradient is an ordinary
// convolution of the output gradient.
template <int DT>
__global__ void k_pack(const float *__restrict__ w, int Cout, int Cin, int k, int n_pad, int cin_pad,
                       int mode, typename Elem<DT>::T *__restrict__ dst) {
    const int tap_split = mode == 1;
    const int taps = tap_split ? 1 : k * k;
    const size_t total = (size_t)taps * n_pad * cin_pad;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % cin_pad);
        const int n = (int)((e / cin_pad) % n_pad);
        const int tap = (int)(e / ((size_t)cin_pad * n_pad));
        float val = 0.f;
        if (tap_split) {
            // one output row per source tap of the single-output layer
            if (n < k * k && c < Cin) val = w[(size_t)c * k * k + n];
        } else if (mode == 2) {
            // n runs over the layer's inputs, c over its outputs
            if (n < Cin && c < Cout) val = w[((size_t)c * Cin + n) * k * k + (k * k - 1 - tap)];
        } else if (n < Cout && c < Cin) {
            val = w[((size_t)n * Cin + c) * k * k + tap];
        }
        dst[e] = Elem<DT>::make(val);
    }
}

sv_status launch_pack(int dtype, const float *w, int Cout, int Cin, int k, int n_pad, int cin_pad,
                      int tap_split, void *dst, hipStream_t s) {
    const size_t total = (size_t)(tap_split == 1 ? 1 : k * k) * n_pad * cin_pad;
    const int blocks = (int)((total + 255) / 256 < 1024 ? (total + 255) / 256 : 1024);
    switch (dtype) {
    case SV_F32:
        hipLaunchKernelGGL(k_pack<SV_F32>, dim3(blocks), dim3(256), 0, s, w, Cout, Cin, k, n_pad,
                           cin_pad, tap_split, (float *)dst);
        break;
    case SV_BF16:
        hipLaunchKernelGGL(k_pack<SV_BF16>, dim3(blocks), dim3(256), 0, s, w, Cout, Cin, k, n_pad,
                           cin_pad, tap_split, (uint16_t *)dst);
        break;
    case SV_F16:
        hipLaunchKernelGGL(k_pack<SV_F16>, dim3(blocks), dim3(256), 0, s, w, Cout, Cin, k, n_pad,
                           cin_pad, tap_split, (uint16_t *)dst);
        break;
    default:
        return SV_ERR_DTYPE;
    }
    SV_LAUNCH_CHECK("k_pack");
    return SV_OK;
}

// INT8 packing: one workgroup per output row n.  a = max |w[n]| over its
// inputs and taps (FP32), code = clamp(rint(w * (127 / a)), -127, 127),
// scale = a / 127; rows past Cout and columns past Cin are 0.
__global__ void __launch_bounds__(256)
k_pack_i8(const float *__restrict__ w, int Cout, int Cin, int k, int n_pad, int cin_pad, int8_t *__restrict__ dst,
          float *__restrict__ scale) {
    __shared__ float red[256];
    const int n = blockIdx.x;
    const int taps = k * k, len = Cin * taps;
    float m = 0.f;
    if (n < Cout)
        for (int e = threadIdx.x; e < len; e += 256) m = fmaxf(m, fabsf(w[(size_t)n * len + e]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const float a = red[0];
    const float inv = a > 0.f ? 127.0f / a : 0.f;
    if (threadIdx.x == 0) scale[n] = n < Cout ? a / 127.0f : 0.f;
    for (int e = threadIdx.x; e < taps * cin_pad; e += 256) {
        const int tap = e / cin_pad, c = e - tap * cin_pad;
        const float v = (n < Cout && c < Cin) ? w[((size_t)n * Cin + c) * taps + tap] : 0.f;
        dst[((size_t)tap * n_pad + n) * cin_pad + c] = quant_i8(v, inv);
    }
}

sv_status launch_pack_i8(const float *w, int Cout, int Cin, int k, int n_pad, int cin_pad, int8_t *dst,
                         float *scale, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_i8, dim3(n_pad), dim3(256), 0, s, w, Cout, Cin, k, n_pad, cin_pad, dst, scale);
    SV_LAUNCH_CHECK("k_pack_i8");
    return SV_OK;
}

__global__ void k_amax_zero(uint32_t *__restrict__ amax, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) amax[i] = 0u;
}

// max(scale0 * d, img / 256) over the coarse pixels, one slot word per workgroup
__global__ void __launch_bounds__(256)
k_amax_x0(uint32_t *__restrict__ slot, const uint8_t *__restrict__ disp, const uint8_t *__restrict__ img,
          long long n, float scale0) {
    float m = 0.f;
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        m = fmaxf(m, fmaxf(scale0 * (float)disp[i], (float)img[i] * (1.0f / 256.0f)));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) atomicMax(slot + (blockIdx.x & (AMAX_SUB - 1)), __float_as_uint(m));
}

sv_status launch_amax_prologue(uint32_t *amax, int nslots, int x0_slot, const uint8_t *disp,
                               const uint8_t *img, long long n, float scale0, hipStream_t s) {
    const int nw = nslots * AMAX_SUB;
    hipLaunchKernelGGL(k_amax_zero, dim3(cdiv(nw, 256)), dim3(256), 0, s, amax, nw);
    SV_LAUNCH_CHECK("k_amax_zero");
    const int blocks = (int)std::min<long long>((n + 255) / 256, 256);
    hipLaunchKernelGGL(k_amax_x0, dim3(blocks), dim3(256), 0, s, amax + (size_t)x0_slot * AMAX_SUB, disp, img, n,
                       scale0);
    SV_LAUNCH_CHECK("k_amax_x0");
    return SV_OK;
}

}  // namespace sv
