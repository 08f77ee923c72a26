// Implicit-GEMM convolution kernel templates (included by the per-dtype
// instantiation files conv_f32.hip, conv_bf16.hip, conv_f16.hip).
#pragma once

#include "kernels.h"

// The tile configurations: (index, TH rows, TN output channels, WM waves along
// rows, KCM base channel chunks staged at once, FB batched staging, name).
#define SV_CONV_CFGS(X)                          \
    X(0, 4, 64, 4, 1, 0, "th4_tn64")             \
    X(1, 8, 64, 4, 1, 0, "th8_tn64")             \
    X(2, 4, 32, 4, 1, 0, "th4_tn32")             \
    X(3, 8, 32, 4, 1, 0, "th8_tn32")             \
    X(4, 2, 64, 2, 1, 0, "th2_tn64")             \
    X(5, 4, 16, 4, 1, 0, "th4_tn16")             \
    X(6, 4, 16, 4, 4, 0, "th4_tn16_k4")          \
    X(7, 4, 32, 4, 2, 0, "th4_tn32_k2")          \
    X(8, 4, 16, 4, 2, 0, "th4_tn16_k2")          \
    X(9, 8, 16, 4, 2, 0, "th8_tn16_k2")          \
    X(10, 4, 64, 4, 2, 0, "th4_tn64_k2")         \
    X(11, 4, 16, 4, 1, 1, "th4_tn16_b")          \
    X(12, 4, 16, 4, 2, 1, "th4_tn16_k2_b")       \
    X(13, 4, 16, 4, 4, 1, "th4_tn16_k4_b")       \
    X(14, 4, 32, 4, 1, 1, "th4_tn32_b")          \
    X(15, 4, 64, 4, 1, 1, "th4_tn64_b")          \
    X(16, 2, 64, 2, 1, 1, "th2_tn64_b")

namespace sv {

template <int DT> struct Mfma;

template <> struct Mfma<SV_BF16> {
    static constexpr int GS = 8;  // k values per lane per step
    typedef uint16_t T;
    typedef u16x8 vec;
    static __device__ __forceinline__ f32x4 run(vec a, vec b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
};

template <> struct Mfma<SV_F16> {
    static constexpr int GS = 8;
    typedef uint16_t T;
    typedef u16x8 vec;
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
    static __device__ __forceinline__ f32x4 run(vec a, vec b, f32x4 c) {
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
        return c;
    }
};

// Converts GS FP32 values into one storage vector.
template <int DT, int GS>
__device__ __forceinline__ typename Mfma<DT>::vec pack_vec(const float (&v)[GS]) {
    typename Mfma<DT>::vec r;
#pragma unroll
    for (int i = 0; i < GS; ++i) r[i] = Elem<DT>::make(v[i]);
    return r;
}

// Reads GS consecutive channels of one pixel of a stored NHWC map into FP32;
// sdt is the map's storage dtype (SV_F32, SV_BF16 or SV_F16).
template <int DT, int GS>
__device__ __forceinline__ void load_px(const void *base, size_t off, int sdt, float (&v)[GS]) {
    if (sdt == SV_F32) {
        const float *p = (const float *)base + off;
#pragma unroll
        for (int i = 0; i < GS; i += 4) {
            f32x4 q = *(const f32x4 *)(p + i);
            v[i] = q[0]; v[i + 1] = q[1]; v[i + 2] = q[2]; v[i + 3] = q[3];
        }
    } else {
        const uint16_t *p = (const uint16_t *)base + off;
        uint16_t h[GS];
        if (GS == 8) {
            const u16x8 q = *(const u16x8 *)p;
#pragma unroll
            for (int i = 0; i < GS; ++i) h[i] = q[i];
        } else {
            const u16x4 q = *(const u16x4 *)p;
#pragma unroll
            for (int i = 0; i < GS; ++i) h[i] = q[i];
        }
#pragma unroll
        for (int i = 0; i < GS; ++i) v[i] = sdt == SV_BF16 ? bf16_bits_to_f32(h[i]) : f16_bits_to_f32(h[i]);
    }
}

// Where one tile's data lives: sizes of the input and output grids, the pixel
// offset of the image in each source and in the output, and the tile origin.
struct ConvGeo {
    int Hi, Wi, Ho, Wo;
    long long sbase[2];
    int hs[2], ws[2];
    long long obase;
    int n0, oy0, ox0;
};

template <int DT, int KS, int S, int TH, int TN, int WM, int KCM, int FB>
struct ConvTile {
    using M = Mfma<DT>;
    using T = typename M::T;
    using vec = typename M::vec;
    static constexpr int GS = M::GS;
    static constexpr int TW = 16;
    static constexpr int TAPS = KS * KS;
    static constexpr int PAD = (KS - 1) / 2;
    static constexpr int PH = (TH - 1) * S + KS, PW = (TW - 1) * S + KS;
    // The reduction runs over base chunks of KCB channels in a fixed order; a
    // tile stages KCM base chunks at once (fewer round trips to memory) but
    // consumes them in the same order, so results do not depend on KCM.
    static constexpr int KCB = DT == SV_F32 ? 16 : 32;
    static constexpr int KC = KCB * KCM;
    static constexpr int KCG = KC / GS;
    static constexpr int KCGB = KCB / GS;
    static constexpr int KCP = KC + GS;  // padded LDS row, in elements
    static constexpr int WN = 4 / WM;
    static constexpr int MBW = TH / WM;
    static constexpr int NBW = TN / 16 / WN;
    static constexpr int NSTEP = (TAPS * KCGB + 3) / 4;
    static_assert(TH % WM == 0 && (TN / 16) % WN == 0 && KC % GS == 0, "tile");

    struct Smem {
        T patch[PH * PW * KCP];
        T wl[TAPS * TN * KCP];
    };

    // per-thread share of a chunk's staging work
    static constexpr int EP = (PH * PW * KCG + 255) / 256;
    static constexpr int EW = (TAPS * TN * KCG + 255) / 256;

    // One patch vector as fetched from global memory, before conversion.
    enum { R_ZERO = 0, R_RAW, R_F32, R_H16, R_RESIZE, R_RESIZE_CVT, R_X0 };
    // r holds raw bits only (moved, never used in arithmetic before commit):
    // one vector of the compute dtype, 8 FP32 values, 4 resize corners, GS
    // 16-bit values of another dtype, or the two x0 bytes.
    struct PRaw {
        f32x4 r[4];
        float ly, lx;    // resize weights; ly = scale of the disparity byte for x0
        int mode, sdt;   // how to commit; storage dtype for conversions
    };
    static __device__ __forceinline__ float ubits(uint32_t u) { return __builtin_bit_cast(float, u); }
    static __device__ __forceinline__ uint32_t fbits(float f) { return __builtin_bit_cast(uint32_t, f); }

    static __device__ __forceinline__ f32x4 as_f4(vec x) { return __builtin_bit_cast(f32x4, x); }
    static __device__ __forceinline__ vec as_vec(f32x4 x) { return __builtin_bit_cast(vec, x); }

    // Issues the global loads of chunk c0 (no use of the loaded values here).
    static __device__ __forceinline__ void fetch(const ConvParams &p, const ConvGeo &G, int c0,
                                                 PRaw (&pr)[EP], vec (&wr)[EW]) {
        const int tid = threadIdx.x;
        const int iy0 = G.oy0 * S - PAD, ix0 = G.ox0 * S - PAD;
#pragma unroll
        for (int k = 0; k < EP; ++k) {
            const int e = tid + k * 256;
            PRaw &R = pr[k];
            R.mode = R_ZERO;
            if (e >= PH * PW * KCG) continue;
            const int cg = e % KCG, pix = e / KCG;
            const int py = pix / PW, px = pix - py * PW;
            const int yi = iy0 + py, xi = ix0 + px, c = c0 + cg * GS;
            if (!(yi >= 0 && yi < G.Hi && xi >= 0 && xi < G.Wi && c < p.Cin)) continue;
            const int si = c < p.src[0].C ? 0 : 1;
            const ConvSrc &s = p.src[si];
            const int cl = c - (si ? p.src[0].C : 0);
            const int sdt = s.sdt ? s.sdt - 1 : DT;
            const long long sb = G.sbase[si];
            const int hs = G.hs[si], ws = G.ws[si];
            R.sdt = sdt;
            if (s.kind == SRC_TENSOR || s.kind == SRC_ZINS) {
                int yy = yi, xx = xi;
                if (s.kind == SRC_ZINS) {
                    if ((yi | xi) & 1) continue;
                    yy = yi >> 1;
                    xx = xi >> 1;
                }
                const size_t off = (size_t)(sb + (long long)yy * ws + xx) * s.pitch + s.coff + cl;
                if (sdt == DT) {
                    R.r[0] = as_f4(*(const vec *)((const T *)s.ptr + off));
                    R.mode = R_RAW;
                } else if (sdt == SV_F32) {
                    const float *q = (const float *)s.ptr + off;
                    R.r[0] = *(const f32x4 *)q;
                    if (GS == 8) R.r[1] = *(const f32x4 *)(q + 4);
                    R.mode = R_F32;
                } else {  // 16-bit storage of another dtype
                    const uint16_t *q = (const uint16_t *)s.ptr + off;
                    if (GS == 8) {
                        R.r[0] = __builtin_bit_cast(f32x4, *(const u16x8 *)q);
                    } else {
                        const u16x4 hv = *(const u16x4 *)q;
                        R.r[0][0] = ubits((uint32_t)hv[0] | ((uint32_t)hv[1] << 16));
                        R.r[0][1] = ubits((uint32_t)hv[2] | ((uint32_t)hv[3] << 16));
                    }
                    R.mode = R_H16;
                }
            } else if (s.kind == SRC_RESIZE) {
                int y0, y1, x0, x1;
                bilin(yi, hs, G.Hi, y0, y1, R.ly);
                bilin(xi, ws, G.Wi, x0, x1, R.lx);
                const size_t cb = (size_t)s.coff + cl;
                const size_t o[4] = {(size_t)(sb + (long long)y0 * ws + x0) * s.pitch + cb,
                                     (size_t)(sb + (long long)y0 * ws + x1) * s.pitch + cb,
                                     (size_t)(sb + (long long)y1 * ws + x0) * s.pitch + cb,
                                     (size_t)(sb + (long long)y1 * ws + x1) * s.pitch + cb};
                if (sdt == DT) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) R.r[j] = as_f4(*(const vec *)((const T *)s.ptr + o[j]));
                    R.mode = R_RESIZE;
                } else {  // other storage: interpolate now (not on the network's path)
                    float a[4][GS], v[GS];
#pragma unroll
                    for (int j = 0; j < 4; ++j) load_px<DT, GS>(s.ptr, o[j], sdt, a[j]);
#pragma unroll
                    for (int i = 0; i < GS; ++i) {
                        const float top = (1.f - R.lx) * a[0][i] + R.lx * a[1][i];
                        const float bot = (1.f - R.lx) * a[2][i] + R.lx * a[3][i];
                        v[i] = (1.f - R.ly) * top + R.ly * bot;
                    }
                    R.r[0] = as_f4(pack_vec<DT, GS>(v));
                    R.mode = R_RESIZE_CVT;
                }
            } else {  // SRC_X0: the two bytes, converted at commit
                const size_t o = (size_t)(sb + (long long)yi * ws + xi);
                R.ly = s.scale0;
                R.r[0][0] = ubits(((const uint8_t *)s.ptr)[o]);
                R.r[0][1] = ubits(s.img[o]);
                R.mode = R_X0;
            }
        }
        const T *wpk = (const T *)p.wpk;
#pragma unroll
        for (int k = 0; k < EW; ++k) {
            const int e = tid + k * 256;
#pragma unroll
            for (int i = 0; i < GS; ++i) wr[k][i] = 0;
            if (e >= TAPS * TN * KCG) continue;
            const int cg = e % KCG, r = e / KCG;
            const int n = r % TN, tap = r / TN;
            const int c = c0 + cg * GS, ng = G.n0 + n;
            if (ng < p.n_pad && c < p.cin_pad)
                wr[k] = *(const vec *)(wpk + ((size_t)tap * p.n_pad + ng) * p.cin_pad + c);
        }
    }

    // Converts the fetched values and writes them to LDS.
    static __device__ __forceinline__ void commit(const PRaw (&pr)[EP], const vec (&wr)[EW], T *patch,
                                                  T *wl) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int k = 0; k < EP; ++k) {
            const int e = tid + k * 256;
            if (e >= PH * PW * KCG) continue;
            const PRaw &R = pr[k];
            const int cg = e % KCG, pix = e / KCG;
            vec out;
            float v[GS];
            switch (R.mode) {
            case R_RAW:
            case R_RESIZE_CVT:
                out = as_vec(R.r[0]);
                break;
            case R_F32:
#pragma unroll
                for (int i = 0; i < GS; ++i) v[i] = i < 4 ? R.r[0][i] : R.r[1][i - 4];
                out = pack_vec<DT, GS>(v);
                break;
            case R_H16:
#pragma unroll
                for (int i = 0; i < GS; ++i) {
                    const uint16_t h = (uint16_t)(fbits(R.r[0][i >> 1]) >> (16 * (i & 1)));
                    v[i] = R.sdt == SV_BF16 ? bf16_bits_to_f32(h) : f16_bits_to_f32(h);
                }
                out = pack_vec<DT, GS>(v);
                break;
            case R_RESIZE: {
                const vec a00 = as_vec(R.r[0]), a01 = as_vec(R.r[1]), a10 = as_vec(R.r[2]),
                          a11 = as_vec(R.r[3]);
#pragma unroll
                for (int i = 0; i < GS; ++i) {
                    const float top = (1.f - R.lx) * Elem<DT>::load((const T *)&a00 + i) +
                                      R.lx * Elem<DT>::load((const T *)&a01 + i);
                    const float bot = (1.f - R.lx) * Elem<DT>::load((const T *)&a10 + i) +
                                      R.lx * Elem<DT>::load((const T *)&a11 + i);
                    v[i] = (1.f - R.ly) * top + R.ly * bot;
                }
                out = pack_vec<DT, GS>(v);
                break;
            }
            case R_X0:
#pragma unroll
                for (int i = 0; i < GS; ++i) v[i] = 0.f;
                v[0] = R.ly * (float)fbits(R.r[0][0]);
                v[1] = (float)fbits(R.r[0][1]) * (1.0f / 256.0f);
                out = pack_vec<DT, GS>(v);
                break;
            default:
#pragma unroll
                for (int i = 0; i < GS; ++i) out[i] = 0;
            }
            *(vec *)&patch[pix * KCP + cg * GS] = out;
        }
#pragma unroll
        for (int k = 0; k < EW; ++k) {
            const int e = tid + k * 256;
            if (e >= TAPS * TN * KCG) continue;
            const int cg = e % KCG, r = e / KCG;
            const int n = r % TN, tap = r / TN;
            *(vec *)&wl[(tap * TN + n) * KCP + cg * GS] = wr[k];
        }
    }

    static __device__ __forceinline__ void run(const ConvParams &p, const ConvGeo &G, Smem &sm) {
        T *patch = sm.patch, *wl = sm.wl;
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int wm = wave % WM, wn = wave / WM;
        const int n0 = G.n0, ox0 = G.ox0, oy0 = G.oy0;
        const int iy0 = oy0 * S - PAD, ix0 = ox0 * S - PAD;
        const int g = lane >> 4, r16 = lane & 15;

        f32x4 acc[MBW][NBW];
#pragma unroll
        for (int i = 0; i < MBW; ++i)
#pragma unroll
            for (int j = 0; j < NBW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

        const T *wpk = (const T *)p.wpk;
        for (int c0 = 0; c0 < p.Cin; c0 += KC) {
          if constexpr (FB) {
            // batched staging: every global load of the chunk is issued first,
            // then converted / interpolated and written to LDS
            PRaw pr[EP];
            vec wr[EW];
            fetch(p, G, c0, pr, wr);
            __syncthreads();  // the previous chunk's MFMAs are done with LDS
            commit(pr, wr, patch, wl);
            __syncthreads();
          } else {
            // serial staging: one element at a time (fewest registers)
            __syncthreads();
            // ---- input patch ------------------------------------------------------
            for (int e = tid; e < PH * PW * KCG; e += 256) {
                const int cg = e % KCG, pix = e / KCG;
                const int py = pix / PW, px = pix - py * PW;
                const int yi = iy0 + py, xi = ix0 + px, c = c0 + cg * GS;
                vec out;
#pragma unroll
                for (int i = 0; i < GS; ++i) out[i] = 0;
                if (yi >= 0 && yi < G.Hi && xi >= 0 && xi < G.Wi && c < p.Cin) {
                    const int si = c < p.src[0].C ? 0 : 1;
                    const ConvSrc &s = p.src[si];
                    const int cl = c - (si ? p.src[0].C : 0);
                    const int sdt = s.sdt ? s.sdt - 1 : DT;
                    const bool raw = sdt == DT;
                    const long long sb = G.sbase[si];
                    const int hs = G.hs[si], ws = G.ws[si];
                    float v[GS];
                    if (s.kind == SRC_TENSOR) {
                        const size_t off = (size_t)(sb + (long long)yi * ws + xi) * s.pitch + s.coff + cl;
                        if (raw) {
                            out = *(const vec *)((const T *)s.ptr + off);
                        } else {
                            load_px<DT, GS>(s.ptr, off, sdt, v);
                            out = pack_vec<DT, GS>(v);
                        }
                    } else if (s.kind == SRC_RESIZE) {
                        int y0, y1, x0, x1;
                        float ly, lx;
                        bilin(yi, hs, G.Hi, y0, y1, ly);
                        bilin(xi, ws, G.Wi, x0, x1, lx);
                        float a00[GS], a01[GS], a10[GS], a11[GS];
                        const size_t cb = (size_t)s.coff + cl;
                        load_px<DT, GS>(s.ptr, (size_t)(sb + (long long)y0 * ws + x0) * s.pitch + cb, sdt, a00);
                        load_px<DT, GS>(s.ptr, (size_t)(sb + (long long)y0 * ws + x1) * s.pitch + cb, sdt, a01);
                        load_px<DT, GS>(s.ptr, (size_t)(sb + (long long)y1 * ws + x0) * s.pitch + cb, sdt, a10);
                        load_px<DT, GS>(s.ptr, (size_t)(sb + (long long)y1 * ws + x1) * s.pitch + cb, sdt, a11);
#pragma unroll
                        for (int i = 0; i < GS; ++i) {
                            const float top = (1.f - lx) * a00[i] + lx * a01[i];
                            const float bot = (1.f - lx) * a10[i] + lx * a11[i];
                            v[i] = (1.f - ly) * top + ly * bot;
                        }
                        out = pack_vec<DT, GS>(v);
                    } else if (s.kind == SRC_ZINS) {
                        if (((yi | xi) & 1) == 0) {
                            const size_t off =
                                (size_t)(sb + (long long)(yi >> 1) * ws + (xi >> 1)) * s.pitch + s.coff + cl;
                            if (raw) {
                                out = *(const vec *)((const T *)s.ptr + off);
                            } else {
                                load_px<DT, GS>(s.ptr, off, sdt, v);
                                out = pack_vec<DT, GS>(v);
                            }
                        }
                    } else {  // SRC_X0: [f*d/256, I/256]
                        const size_t o = (size_t)(sb + (long long)yi * ws + xi);
#pragma unroll
                        for (int i = 0; i < GS; ++i) v[i] = 0.f;
                        v[0] = s.scale0 * (float)((const uint8_t *)s.ptr)[o];
                        v[1] = (float)s.img[o] * (1.0f / 256.0f);
                        out = pack_vec<DT, GS>(v);
                    }
                }
                *(vec *)&patch[(py * PW + px) * KCP + cg * GS] = out;
            }
            // ---- weights ------------------------------------------------------------
            for (int e = tid; e < TAPS * TN * KCG; e += 256) {
                const int cg = e % KCG, r = e / KCG;
                const int n = r % TN, tap = r / TN;
                const int c = c0 + cg * GS, ng = n0 + n;
                vec val;
#pragma unroll
                for (int i = 0; i < GS; ++i) val[i] = 0;
                if (ng < p.n_pad && c < p.cin_pad)
                    val = *(const vec *)(wpk + ((size_t)tap * p.n_pad + ng) * p.cin_pad + c);
                *(vec *)&wl[(tap * TN + n) * KCP + cg * GS] = val;
            }
            __syncthreads();
          }
            // ---- MFMA over (tap, channel-group) pairs, base chunk by base chunk --
#pragma unroll
            for (int sub = 0; sub < KCM; ++sub) {
            if (c0 + sub * KCB >= p.Cin) break;
            // unrolled so the LDS operand loads of later steps are issued ahead
            // of the MFMAs of earlier ones
#pragma unroll
            for (int st = 0; st < NSTEP; ++st) {
                const int q = st * 4 + g;
                const bool valid = q < TAPS * KCGB;
                const int tap = valid ? q / KCGB : 0;
                const int cg = sub * KCGB + (valid ? q % KCGB : 0);
                const int u = tap / KS, v = tap - (tap / KS) * KS;
                vec bf[MBW], af[NBW];
#pragma unroll
                for (int mb = 0; mb < MBW; ++mb) {
                    const int ty = wm * MBW + mb;
                    bf[mb] = *(const vec *)&patch[((ty * S + u) * PW + (r16 * S + v)) * KCP + cg * GS];
                    if (!valid) {
#pragma unroll
                        for (int i = 0; i < GS; ++i) bf[mb][i] = 0;
                    }
                }
#pragma unroll
                for (int nb = 0; nb < NBW; ++nb) {
                    const int n = (wn * NBW + nb) * 16 + r16;
                    af[nb] = *(const vec *)&wl[(tap * TN + n) * KCP + cg * GS];
                }
#pragma unroll
                for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NBW; ++nb) acc[mb][nb] = M::run(af[nb], bf[mb], acc[mb][nb]);
            }
            }
        }

        // ---- epilogue: bias, activation, backward terms, NHWC store ------------
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb) {
            const int oy = oy0 + wm * MBW + mb, ox = ox0 + r16;
            if (oy >= G.Ho || ox >= G.Wo) continue;
            const size_t pix = (size_t)(G.obase + (long long)oy * G.Wo + ox);
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
                const int nbase = n0 + (wn * NBW + nb) * 16 + 4 * g;
                float r[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int n = nbase + i;
                    float val = acc[mb][nb][i] + ((p.bias && n < p.Cout) ? p.bias[n] : 0.f);
                    if (p.act) val = val > 0.f ? val : 0.1f * val;
                    if (n < p.Cout) {
                        if (p.add) val += p.add[pix * p.add_pitch + p.add_coff + n];
                        if (p.mask) {
                            const float mv = Elem<DT>::load((const T *)p.mask + pix * p.mask_pitch + n);
                            val *= mv > 0.f ? 1.0f : 0.1f;
                        }
                    }
                    r[i] = val;
                }
                const size_t o = pix * p.out_pitch + p.out_coff + nbase;
                const bool full = nbase + 4 <= p.Cout;
                if (p.out_f32) {
                    float *op = (float *)p.out + o;
                    if (full && (o % 4) == 0) {
                        *(f32x4 *)op = f32x4{r[0], r[1], r[2], r[3]};
                    } else {
                        for (int i = 0; i < 4; ++i)
                            if (nbase + i < p.Cout) op[i] = r[i];
                    }
                } else {
                    T *op = (T *)p.out + o;
                    if (full && (o % 4) == 0 && DT != SV_F32) {
                        u16x4 w4;
                        for (int i = 0; i < 4; ++i) w4[i] = (uint16_t)Elem<DT>::make(r[i]);
                        *(u16x4 *)op = w4;
                    } else if (full && (o % 4) == 0) {
                        *(f32x4 *)op = f32x4{r[0], r[1], r[2], r[3]};
                    } else {
                        for (int i = 0; i < 4; ++i)
                            if (nbase + i < p.Cout) op[i] = Elem<DT>::make(r[i]);
                    }
                }
            }
        }
    }
};

// Uniform batch: one workgroup per (column tile, row tile, image x channel tile).
template <int DT, int KS, int S, int TH, int TN, int WM, int KCM, int FB>
__global__ void __launch_bounds__(256) k_conv(const ConvParams p)
{
    using CT = ConvTile<DT, KS, S, TH, TN, WM, KCM, FB>;
    __shared__ __attribute__((aligned(16))) typename CT::Smem sm;
    const int ntn = (p.Cout + TN - 1) / TN;
    const int b = blockIdx.z / ntn;
    ConvGeo G;
    G.Hi = p.Hi; G.Wi = p.Wi; G.Ho = p.Ho; G.Wo = p.Wo;
    for (int i = 0; i < 2; ++i) {
        G.hs[i] = p.src[i].hs;
        G.ws[i] = p.src[i].ws;
        G.sbase[i] = (long long)b * p.src[i].hs * p.src[i].ws;
    }
    G.obase = (long long)b * p.Ho * p.Wo;
    G.n0 = (blockIdx.z % ntn) * TN;
    G.oy0 = blockIdx.y * TH;
    G.ox0 = blockIdx.x * CT::TW;
    CT::run(p, G, sm);
}

// Pair table: persistent loop over the stage's tiles of every pair.
template <int DT, int KS, int S, int TH, int TN, int WM, int KCM, int FB>
__global__ void __launch_bounds__(256) k_conv_tab(const ConvParams p)
{
    using CT = ConvTile<DT, KS, S, TH, TN, WM, KCM, FB>;
    __shared__ __attribute__((aligned(16))) typename CT::Smem sm;
    const PairTable *tab = p.tab;
    const int n = tab->n;
    const int *cum = tab->cum[p.stage];
    const int total = cum[n];
    const int ntn = (p.Cout + TN - 1) / TN;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = table_find(cum, n, t);
        const PairGeo &pg = tab->pair[i];
        ConvGeo G;
        G.Hi = pg.h[p.in_level]; G.Wi = pg.w[p.in_level];
        G.Ho = pg.h[p.out_level]; G.Wo = pg.w[p.out_level];
        for (int k = 0; k < 2; ++k) {
            const int lv = p.src[k].level;
            G.hs[k] = pg.h[lv];
            G.ws[k] = pg.w[lv];
            G.sbase[k] = pg.off[lv];
        }
        G.obase = pg.off[p.out_level];
        const int local = t - cum[i];
        const int tx = cdiv_d(G.Wo, CT::TW), ty = cdiv_d(G.Ho, TH);
        const int nt = local / (tx * ty), r = local - nt * tx * ty;
        G.n0 = nt * TN;
        G.oy0 = (r / tx) * TH;
        G.ox0 = (r % tx) * CT::TW;
        CT::run(p, G, sm);
        (void)ntn;
    }
}

// grid <= 0: uniform launch; grid > 0: persistent launch over p.tab.
template <int DT, int KS, int S, int TH, int TN, int WM, int KCM, int FB>
static sv_status launch_one(const ConvParams &p, int pgrid, hipStream_t st) {
    if (pgrid > 0) {
        hipLaunchKernelGGL((k_conv_tab<DT, KS, S, TH, TN, WM, KCM, FB>), dim3(pgrid), dim3(256), 0, st, p);
        SV_LAUNCH_CHECK("k_conv_tab");
        return SV_OK;
    }
    dim3 grid(cdiv(p.Wo, 16), cdiv(p.Ho, TH), p.B * cdiv(p.Cout, TN));
    hipLaunchKernelGGL((k_conv<DT, KS, S, TH, TN, WM, KCM, FB>), grid, dim3(256), 0, st, p);
    SV_LAUNCH_CHECK("k_conv");
    return SV_OK;
}

template <int DT, int KS, int S>
static sv_status launch_cfg(int cfg, const ConvParams &p, int pg, hipStream_t st) {
    switch (cfg) {
#define SV_CFG(i, TH, TN, WM, KCM, FB, name) \
    case i: return launch_one<DT, KS, S, TH, TN, WM, KCM, FB>(p, pg, st);
        SV_CONV_CFGS(SV_CFG)
#undef SV_CFG
    default: return SV_ERR_RANGE;
    }
}

template <int DT>
static sv_status launch_dt(int ks, int stride, int cfg, const ConvParams &p, int pg, hipStream_t st) {
    if (ks == 3 && stride == 1) return launch_cfg<DT, 3, 1>(cfg, p, pg, st);
    if (ks == 3 && stride == 2) return launch_cfg<DT, 3, 2>(cfg, p, pg, st);
    if (ks == 1 && stride == 1) return launch_cfg<DT, 1, 1>(cfg, p, pg, st);
    return SV_ERR_UNSUPPORTED;
}


}  // namespace sv
