// Implicit-GEMM convolution kernel templates (included by the per-dtype
// instantiation files conv_f32.hip, conv_bf16.hip, conv_f16.hip, and by
// conv5_<stride>_<dtype>.hip for 5x5 kernels).
#pragma once

#include <algorithm>

#include "kernels.h"
#include "mfma.h"

// The tile configurations: (index, TH rows, TN output channels, WM waves along
// rows, KCM base channel chunks staged at once, name).
#define SV_CONV_CFGS(X)                    \
    X(0, 4, 64, 4, 1, "th4_tn64")          \
    X(1, 8, 64, 4, 1, "th8_tn64")          \
    X(2, 4, 32, 4, 1, "th4_tn32")          \
    X(3, 8, 32, 4, 1, "th8_tn32")          \
    X(4, 2, 64, 2, 1, "th2_tn64")          \
    X(5, 4, 16, 4, 1, "th4_tn16")          \
    X(6, 4, 16, 4, 4, "th4_tn16_k4")       \
    X(7, 4, 32, 4, 2, "th4_tn32_k2")       \
    X(8, 4, 16, 4, 2, "th4_tn16_k2")       \
    X(9, 8, 16, 4, 2, "th8_tn16_k2")       \
    X(10, 4, 64, 4, 2, "th4_tn64_k2")      \
    X(11, 2, 32, 2, 2, "th2_tn32_k2")      \
    X(12, 2, 64, 2, 2, "th2_tn64_k2")      \
    X(13, 4, 16, 4, 8, "th4_tn16_k8")      \
    X(14, 2, 32, 2, 4, "th2_tn32_k4")      \
    X(15, 4, 32, 4, 4, "th4_tn32_k4")      \
    X(16, 16, 32, 4, 1, "th16_tn32")

namespace sv {

// Storage dtype of a compute dtype's activations: INT8 layers keep BF16 maps.
template <int DT> struct Store { static constexpr int v = DT; };
template <> struct Store<SV_I8> { static constexpr int v = SV_BF16; };

// INT8 code of an FP32 value for a tensor quantised with 127 / amax = qinv.
__device__ __forceinline__ int8_t quant_i8(float v, float qinv) {
    const float q = fminf(fmaxf(rintf(v * qinv), -127.0f), 127.0f);
    return (int8_t)(int)q;
}

// Converts GS FP32 values into one LDS vector of the compute dtype (INT8:
// quantised with qinv, ignored otherwise).
template <int DT, int GS>
__device__ __forceinline__ typename Mfma<DT>::vec pack_vec(const float (&v)[GS], float qinv) {
    typename Mfma<DT>::vec r;
    if constexpr (DT == SV_I8) {
#pragma unroll
        for (int i = 0; i < GS; ++i) r[i] = quant_i8(v[i], qinv);
    } else if constexpr (DT == SV_BF16) {
        // two values per v_cvt_pk_bf16_f32 (round to nearest even, as Elem::make)
        typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
        typedef float f32x2_t __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int i = 0; i < GS; i += 2) {
            const bf16x2_t h = __builtin_convertvector((f32x2_t){v[i], v[i + 1]}, bf16x2_t);
            const uint32_t u = __builtin_bit_cast(uint32_t, h);
            r[i] = (uint16_t)(u & 0xffffu);
            r[i + 1] = (uint16_t)(u >> 16);
        }
    } else {
#pragma unroll
        for (int i = 0; i < GS; ++i) r[i] = Elem<DT>::make(v[i]);
    }
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

// Epilogue of four consecutive output channels nbase..nbase+3 of one output
// pixel from their FP32 sums: bias, activation, the backward pass's extra
// terms, then an NHWC store in the output dtype.
template <int DT>
__device__ __forceinline__ void conv_bias4(const ConvParams &p, int nbase, float (&b)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = (p.bias && nbase + i < p.Cout) ? p.bias[nbase + i] : 0.f;
}

// Returns max |stored value| over the channels it wrote (for amax_out).
template <int DT0>
__device__ __forceinline__ float conv_epilogue(const ConvParams &p, size_t pix, int nbase,
                                               const float (&acc)[4], const float (&bias)[4]) {
    constexpr int DT = Store<DT0>::v;
    using T = typename Elem<DT>::T;
    float r[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int n = nbase + i;
        float val = acc[i] + bias[i];
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
    float amax = 0.f;
    if (p.out_f32) {
        float *op = (float *)p.out + o;
        if (full && (o % 4) == 0) {
            *(f32x4 *)op = f32x4{r[0], r[1], r[2], r[3]};
        } else {
            for (int i = 0; i < 4; ++i)
                if (nbase + i < p.Cout) op[i] = r[i];
        }
        for (int i = 0; i < 4; ++i)
            if (nbase + i < p.Cout) amax = fmaxf(amax, fabsf(r[i]));
    } else {
        T *op = (T *)p.out + o;
        T st[4];
        for (int i = 0; i < 4; ++i) {
            st[i] = Elem<DT>::make(r[i]);
            if (nbase + i < p.Cout) amax = fmaxf(amax, fabsf(Elem<DT>::load(&st[i])));
        }
        if (full && (o % 4) == 0 && DT != SV_F32) {
            u16x4 w4;
            for (int i = 0; i < 4; ++i) w4[i] = (uint16_t)st[i];
            *(u16x4 *)op = w4;
        } else if (full && (o % 4) == 0) {
            *(f32x4 *)op = f32x4{r[0], r[1], r[2], r[3]};
        } else {
            for (int i = 0; i < 4; ++i)
                if (nbase + i < p.Cout) op[i] = st[i];
        }
    }
    return amax;
}

// Adds one workgroup's output maximum to amax_out: a wave-wide max, then one
// vector atomic per wave into the workgroup's slot.
__device__ __forceinline__ void record_amax(const ConvParams &p, float m, int slot) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) atomicMax(p.amax_out + (slot & (AMAX_SUB - 1)), __float_as_uint(m));
}

// The same with one atomic per workgroup of four waves: the waves' maxima
// meet in red[4] (LDS); every thread of the workgroup calls it.  Atomics to
// one slot serialise, so a quarter of them shortens layers with many
// workgroups.
__device__ __forceinline__ void record_amax_wg(const ConvParams &p, float m, int slot, float *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(p.amax_out + (slot & (AMAX_SUB - 1)),
                  __float_as_uint(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]))));
}

// The input scale of an INT8 layer: m = the largest recorded amax of its
// sources; qinv = 127 / m and s_in = m / 127 (both 0 when m = 0).  Lane j
// reads word j of each source's slots, then a wave-wide max.
__device__ __forceinline__ void input_scale(const ConvParams &p, float &qinv, float &s_in) {
    const int lane = threadIdx.x & 63;
    float m = 0.f;
    for (int k = 0; k < 2; ++k)
        if (p.amax_in[k]) m = fmaxf(m, __uint_as_float(p.amax_in[k][lane]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    qinv = m > 0.f ? 127.0f / m : 0.f;
    s_in = m / 127.0f;
}

// The range [c_begin, c_end) of input channels that reduction part kz of
// ksplit covers: ksplit contiguous runs of base chunks of kcb channels, the
// same for every tile shape.
__device__ __forceinline__ void split_range(int Cin, int kcb, int ksplit, int kz, int &c_begin,
                                            int &c_end) {
    const int nb = (Cin + kcb - 1) / kcb;
    const int per = (nb + ksplit - 1) / ksplit;
    c_begin = min(kz * per, nb) * kcb;
    c_end = min(min((kz + 1) * per, nb) * kcb, Cin);
}

// Where one tile's data lives: sizes of the input and output grids, the pixel
// offset of the image in each source and in the output, and the tile origin.
struct ConvGeo {
    int Hi, Wi, Ho, Wo;
    long long sbase[2];
    int hs[2], ws[2];
    long long obase;
    int n0, oy0, ox0, b;
};

template <int DT, int KS, int S, int TH, int TN, int WM, int KCM>
struct ConvTile {
    using M = Mfma<DT>;
    using T = typename M::T;
    using vec = typename M::vec;
    static constexpr int GS = M::GS;
    // storage of the maps this layer reads in its own dtype, and a vector of GS of them
    static constexpr int SD = Store<DT>::v;
    using ST = typename Elem<SD>::T;
    using SVec = typename Mfma<SD>::vec;
    static constexpr int TW = 16;
    static constexpr int TAPS = KS * KS;
    static constexpr int PAD = (KS - 1) / 2;
    static constexpr int PH = (TH - 1) * S + KS, PW = (TW - 1) * S + KS;
    static constexpr int NPIX = PH * PW;
    // The reduction runs over base chunks of KCB channels in a fixed order; a
    // tile stages KCM base chunks at once but consumes them in the same order,
    // so results do not depend on KCM.
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

    // Where a patch pixel reads each source: pixel indices (p[0] < 0: zero
    // padding) of the pixel, or of the four bilinear corners and their weights.
    struct PixSrc {
        int p[4];
        float ly, lx;
    };

    // One axis of the table: the source row (column) pair and weight of each
    // patch row (column); i0 < 0 outside the input grid or on an inserted zero.
    struct AxSrc {
        int i0, i1;
        float lam;
    };

    struct Smem {
        T patch[NPIX * KCP];
        T wl[TAPS * TN * KCP];
        PixSrc ps[2][NPIX];
        AxSrc ax[2][PH + PW];
        float red[4];  // the waves' output maxima (INT8)
    };
    // tiles whose LDS exceeds a CU's 160 KB are never instantiated (conv_fits)
    static constexpr bool FITS = sizeof(Smem) <= 160 * 1024;

    // Computed once per tile; every channel chunk reuses it.  A resized
    // source's index and weight along y depend on the patch row only and along
    // x on the patch column only, so on tiles with more table entries than
    // threads the PH + PW axis entries (with the resize's divisions) are formed
    // first and each pixel combines one of each; otherwise (and for sources
    // read in place, whose entries cost no division) every entry is formed
    // directly, without the second LDS round trip.
    template <bool SEP>
    static __device__ __forceinline__ void pix_table(const ConvParams &p, const ConvGeo &G, Smem &sm) {
        const int iy0 = G.oy0 * S - PAD, ix0 = G.ox0 * S - PAD;
        const bool sep = SEP && 2 * NPIX > 256 && (p.src[0].kind == SRC_RESIZE || p.src[1].kind == SRC_RESIZE);
        if (!sep) {
            for (int e = threadIdx.x; e < 2 * NPIX; e += 256) {
                const int si = e >= NPIX ? 1 : 0, pix = e - si * NPIX;
                const int py = pix / PW, px = pix - py * PW;
                const int yi = iy0 + py, xi = ix0 + px;
                const int kind = si ? p.src[1].kind : p.src[0].kind;
                PixSrc q;
                q.p[0] = q.p[1] = q.p[2] = q.p[3] = -1;
                q.ly = q.lx = 0.f;
                if (kind != SRC_NONE && yi >= 0 && yi < G.Hi && xi >= 0 && xi < G.Wi) {
                    // a pixel index of the batch fits an int (as the table stores it)
                    const int sb = (int)(si ? G.sbase[1] : G.sbase[0]);
                    const int hs = si ? G.hs[1] : G.hs[0], ws = si ? G.ws[1] : G.ws[0];
                    if (kind == SRC_RESIZE) {
                        int y0, y1, x0, x1;
                        bilin(yi, hs, G.Hi, y0, y1, q.ly);
                        bilin(xi, ws, G.Wi, x0, x1, q.lx);
                        q.p[0] = sb + y0 * ws + x0;
                        q.p[1] = sb + y0 * ws + x1;
                        q.p[2] = sb + y1 * ws + x0;
                        q.p[3] = sb + y1 * ws + x1;
                    } else if (kind == SRC_ZINS) {
                        if (((yi | xi) & 1) == 0) q.p[0] = q.p[1] = q.p[2] = q.p[3] = sb + (yi >> 1) * ws + (xi >> 1);
                    } else {
                        q.p[0] = q.p[1] = q.p[2] = q.p[3] = sb + yi * ws + xi;
                    }
                }
                sm.ps[si][pix] = q;
            }
        } else {
            for (int e = threadIdx.x; e < 2 * (PH + PW); e += 256) {
                const int si = e >= PH + PW ? 1 : 0, j = e - si * (PH + PW);
                const bool row = j < PH;
                const int o = row ? iy0 + j : ix0 + (j - PH);
                const int n = row ? G.Hi : G.Wi;
                // one level of selection per value (a nested one would index G in memory)
                const int hsi = si ? G.hs[1] : G.hs[0], wsi = si ? G.ws[1] : G.ws[0];
                const int nin = row ? hsi : wsi;
                const int kind = si ? p.src[1].kind : p.src[0].kind;
                AxSrc a;
                a.i0 = a.i1 = -1;
                a.lam = 0.f;
                if (kind != SRC_NONE && o >= 0 && o < n) {
                    if (kind == SRC_RESIZE) bilin(o, nin, n, a.i0, a.i1, a.lam);
                    else if (kind == SRC_ZINS) a.i0 = a.i1 = (o & 1) == 0 ? o >> 1 : -1;
                    else a.i0 = a.i1 = o;
                }
                sm.ax[si][j] = a;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < 2 * NPIX; e += 256) {
                const int si = e >= NPIX ? 1 : 0, pix = e - si * NPIX;
                const int py = pix / PW, px = pix - py * PW;
                const AxSrc ay = sm.ax[si][py], ax = sm.ax[si][PH + px];
                PixSrc q;
                q.p[0] = q.p[1] = q.p[2] = q.p[3] = -1;
                q.ly = q.lx = 0.f;
                if (ay.i0 >= 0 && ax.i0 >= 0) {
                    const int sb = (int)(si ? G.sbase[1] : G.sbase[0]);
                    const int ws = si ? G.ws[1] : G.ws[0];
                    const int r0 = sb + ay.i0 * ws, r1 = sb + ay.i1 * ws;
                    q.p[0] = r0 + ax.i0;
                    q.p[1] = r0 + ax.i1;
                    q.p[2] = r1 + ax.i0;
                    q.p[3] = r1 + ax.i1;
                    q.ly = ay.lam;
                    q.lx = ax.lam;
                }
                sm.ps[si][pix] = q;
            }
        }
    }

    // Final-layer projection epilogue (see ConvParams::proj_*), itself a small
    // product on the matrix units: T[tap][pixel] = W_F[tap][c] . y[c][pixel]
    // with the nine taps as the rows of A and the wave's 16-pixel blocks as
    // the columns of B.  The wave holds every output channel of its pixels
    // (one channel tile, WN = 1): lane (g, r16) has channels nb * 16 + 4 g + i
    // of pixel r16, so B's k slots of lane group g are exactly those channels
    // and A's rows are built with the same channel order.  FP32 runs the FP32
    // instruction; 16-bit types (and INT8 layers, whose maps are stored as
    // BF16: y is the dequantised sum, biased, activated and rounded to BF16)
    // feed y as stored (exact in the type) and the FP32 weights as a high and
    // a low part, two products in the storage type.  The accumulator
    // comes back as taps 4 g' + i of pixel r16' in lane (g', r16'); the x0
    // terms are added in FP32 and each lane writes its taps.
    static __device__ __forceinline__ void project_epilogue(const ConvParams &p, const ConvGeo &G,
                                                            const typename M::acc (&acc)[MBW][NBW],
                                                            const float (&bpre)[NBW][4],
                                                            const float (&spre)[NBW][4]) {
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int wm = wave % WM;
        const int g = lane >> 4, r16 = lane & 15;
        constexpr int SD = Store<DT>::v;
        const int tap_row = r16 < 9 ? r16 : -1;   // A row = tap
        // A: this lane's weights W_F[tap_row][nb * 16 + 4 g + i]
        float wa[NBW][4];
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) {
            const int n = nb * 16 + 4 * g;
            const bool ok = tap_row >= 0 && n < p.Cout;  // Cout is a multiple of 8: all four or none
            const f32x4 w4 = ok ? *(const f32x4 *)(p.proj_w + tap_row * p.proj_pitch + n) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 4; ++i) wa[nb][i] = w4[i];
        }
        // x0 weights of this lane's output taps 4 g + i
        float wd[4], wi[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = 4 * g + i;
            wd[i] = t < 9 ? p.proj_w[t * p.proj_pitch + p.Cout] : 0.f;
            wi[i] = t < 9 ? p.proj_w[t * p.proj_pitch + p.Cout + 1] : 0.f;
        }
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb) {
            // y as stored, this lane's channels of pixel r16
            float val[NBW][4];
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // (INT8: the integer sum times s_in s_w first, as the plain epilogue)
                    const float a = DT == SV_I8 ? (float)acc[mb][nb][i] * spre[nb][i] : (float)acc[mb][nb][i];
                    float v = a + bpre[nb][i];
                    v = v > 0.f ? v : 0.1f * v;
                    const typename Elem<SD>::T st = Elem<SD>::make(v);
                    val[nb][i] = nb * 16 + 4 * g + i < p.Cout ? Elem<SD>::load(&st) : 0.f;
                }
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            if constexpr (DT == SV_F32) {
#pragma unroll
                for (int nb = 0; nb < NBW; ++nb) {
                    const f32x4 a4 = {wa[nb][0], wa[nb][1], wa[nb][2], wa[nb][3]};
                    const f32x4 b4 = {val[nb][0], val[nb][1], val[nb][2], val[nb][3]};
                    c = M::run(a4, b4, c);
                }
            } else {
#pragma unroll
                for (int pr = 0; pr < (NBW + 1) / 2; ++pr) {
                    float bv[8], ah[8], al[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int nb = 2 * pr + j / 4, i = j % 4;
                        const bool ok = nb < NBW;
                        bv[j] = ok ? val[nb < NBW ? nb : 0][i] : 0.f;
                        const float w = ok ? wa[nb < NBW ? nb : 0][i] : 0.f;
                        const typename Elem<SD>::T wh = Elem<SD>::make(w);
                        ah[j] = Elem<SD>::load(&wh);
                        al[j] = w - ah[j];
                    }
                    using MP = Mfma<SD>;
                    const typename MP::vec bq = pack_vec<SD, 8>(bv, 0.f);
                    c = MP::run(pack_vec<SD, 8>(ah, 0.f), bq, c);
                    c = MP::run(pack_vec<SD, 8>(al, 0.f), bq, c);
                }
            }
            const int oy = G.oy0 + wm * MBW + mb, ox = G.ox0 + r16;
            if (oy >= G.Ho || ox >= G.Wo) continue;
            const size_t pix = (size_t)(G.obase + (long long)oy * G.Wo + ox);
            const float xd = p.proj_scale0 * (float)p.proj_disp[pix];
            const float xi = (float)p.proj_img[pix] * (1.0f / 256.0f);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int t = 4 * g + i;
                if (t < 9) p.proj_out[t * p.proj_plane + pix] = fmaf(wi[i], xi, fmaf(wd[i], xd, c[i]));
            }
        }
    }

    // The x0 chunk: 2 channels x TAPS taps = 2 TAPS values per output pixel,
    // packed into K as k = 2 tap + channel (zeros past 2 TAPS), so the chunk
    // costs ceil(2 TAPS / (4 GS)) MFMA steps instead of TAPS.  The x0 values
    // of the patch are staged as pairs xp[pix][2] (a zero pair after the last
    // pixel serves taps past TAPS), the weights as wx[row][k]; lane group g
    // supplies k = (4 s + g) GS .. + GS - 1 of step s to both operands.
    static constexpr int NKX = 2 * TAPS;
    static constexpr int NSX = (NKX + 4 * GS - 1) / (4 * GS);
    static constexpr int KXP = NSX * 4 * GS + GS;
    static_assert(2 * (NPIX + 1) <= NPIX * KCP && TN * KXP <= TAPS * TN * KCP, "x0 staging fits");

    static __device__ __forceinline__ void x0_packed(const ConvParams &p, Smem &sm,
                                                     typename M::acc (&acc)[MBW][NBW], float qinv,
                                                     int n0, int wm, int wn, int g, int r16) {
        const int tid = threadIdx.x;
        const bool first = p.src[0].kind == SRC_X0;
        const ConvSrc &sx = first ? p.src[0] : p.src[1];
        const PixSrc *tx = sm.ps[first ? 0 : 1];
        const int cx = first ? 0 : p.src[0].C;   // column of x0's first channel in the packed weights
        T *xp = sm.patch, *wx = sm.wl;
        __syncthreads();  // the last chunk's MFMA steps are done with the patch and weights
        for (int pix = tid; pix <= NPIX; pix += 256) {
            const int pi = pix < NPIX ? tx[pix].p[0] : -1;
            float v0 = 0.f, v1 = 0.f;
            if (pi >= 0) {
                v0 = sx.scale0 * (float)((const uint8_t *)sx.ptr)[pi];
                v1 = (float)sx.img[pi] * (1.0f / 256.0f);
            }
            if constexpr (DT == SV_I8) {
                xp[2 * pix] = quant_i8(v0, qinv);
                xp[2 * pix + 1] = quant_i8(v1, qinv);
            } else {
                xp[2 * pix] = Elem<DT>::make(v0);
                xp[2 * pix + 1] = Elem<DT>::make(v1);
            }
        }
        const T *wpk = (const T *)p.wpk;
        for (int e = tid; e < TN * KXP; e += 256) {
            const int n = e / KXP, k = e - n * KXP;
            const int ng = n0 + n;
            T w = (T)0;
            if (k < NKX && ng < p.n_pad) w = wpk[((size_t)(k >> 1) * p.n_pad + ng) * p.cin_pad + cx + (k & 1)];
            wx[e] = w;
        }
        __syncthreads();
#pragma unroll
        for (int st = 0; st < NSX; ++st) {
            vec af[NBW], bf[MBW];
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb)
                af[nb] = *(const vec *)&wx[((wn * NBW + nb) * 16 + r16) * KXP + (st * 4 + g) * GS];
#pragma unroll
            for (int mb = 0; mb < MBW; ++mb) {
                const int ty = wm * MBW + mb;
                const int base = (ty * S) * PW + r16 * S;
#pragma unroll
                for (int m = 0; m < GS / 2; ++m) {
                    const int tap = (st * 4 + g) * (GS / 2) + m;
                    const int u = tap / KS, v = tap - (tap / KS) * KS;
                    const int q = tap < TAPS ? base + u * PW + v : NPIX;
                    // the pair (both channels of one tap) in one LDS read
                    if constexpr (sizeof(T) == 4) {
                        const float2 w2 = *(const float2 *)&xp[2 * q];
                        bf[mb][2 * m] = w2.x;
                        bf[mb][2 * m + 1] = w2.y;
                    } else if constexpr (sizeof(T) == 2) {
                        const uint32_t w2 = *(const uint32_t *)&xp[2 * q];
                        bf[mb][2 * m] = (T)(w2 & 0xffffu);
                        bf[mb][2 * m + 1] = (T)(w2 >> 16);
                    } else {
                        const uint16_t w2 = *(const uint16_t *)&xp[2 * q];
                        bf[mb][2 * m] = (T)(int8_t)(w2 & 0xffu);
                        bf[mb][2 * m + 1] = (T)(int8_t)(w2 >> 8);
                    }
                }
            }
#pragma unroll
            for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
                for (int nb = 0; nb < NBW; ++nb) acc[mb][nb] = M::run(af[nb], bf[mb], acc[mb][nb]);
        }
    }

    template <bool SEP = true>
    static __device__ __forceinline__ void run(const ConvParams &p, const ConvGeo &G, Smem &sm,
                                               int kz) {
        T *patch = sm.patch, *wl = sm.wl;
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int wm = wave % WM, wn = wave / WM;
        const int n0 = G.n0, ox0 = G.ox0, oy0 = G.oy0;
        const int g = lane >> 4, r16 = lane & 15;
        const int C0 = p.src[0].C;

        typename M::acc acc[MBW][NBW];
#pragma unroll
        for (int i = 0; i < MBW; ++i)
#pragma unroll
            for (int j = 0; j < NBW; ++j) acc[i][j] = typename M::acc{0, 0, 0, 0};

        // the bias of this lane's output channels, loaded ahead of the main loop
        float bpre[NBW][4];
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
            conv_bias4<DT>(p, n0 + (wn * NBW + nb) * 16 + 4 * g, bpre[nb]);
        // INT8: the input's quantisation step and, per output channel, the
        // factor s_in * s_w that turns an integer sum into the FP32 value
        float qinv = 0.f, spre[NBW][4];
        if constexpr (DT == SV_I8) {
            float s_in;
            input_scale(p, qinv, s_in);
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int n = n0 + (wn * NBW + nb) * 16 + 4 * g + i;
                    spre[nb][i] = n < p.Cout ? s_in * p.wscale[n] : 0.f;
                }
        }

        __syncthreads();  // the previous tile of a persistent loop is done with LDS
        pix_table<SEP>(p, G, sm);
        const T *wpk = (const T *)p.wpk;
        int c_begin = 0, c_end = p.Cin;
        if (p.ksplit > 1) split_range(p.Cin, KCB, p.ksplit, kz, c_begin, c_end);
        static_assert(KCGB == 4, "a base chunk is four channel groups, one per lane group");
        // The network input x0 (two channels) in a base chunk of its own -- the
        // whole input, or the second source starting on a chunk boundary -- is
        // reduced after the other chunks with its taps packed into K (below);
        // the chunk loop runs up to it.
        int c_x0 = c_end;
        if (p.src[0].kind == SRC_X0 && p.src[1].kind == SRC_NONE) c_x0 = c_begin == 0 ? 0 : c_end;
        else if (p.src[1].kind == SRC_X0 && C0 % KCB == 0 && c_begin <= C0 && C0 < c_end) c_x0 = C0;
        for (int c0 = c_begin; c0 < c_x0; c0 += KC) {
            // base chunks of this round that hold input channels
            const int nsub = min(KCM, (c_x0 - c0 + KCB - 1) / KCB);
            __syncthreads();
            // ---- staging: the input patch (at the precomputed source pixels) and
            // the chunk of weights.  e = pix * KCG + cg and 256 is a multiple of
            // KCG, so a thread keeps one channel group -- one source and one kind
            // -- for the whole chunk.  Loads are issued in branch-free groups
            // (padding and out-of-range elements read a valid address and are
            // zeroed afterwards); each step issues one patch group and one weight
            // group before writing either to LDS, so both are in flight together.
            {
                const int cg = tid % KCG;
                const int c = c0 + cg * GS;
                const int si = c < C0 ? 0 : 1;
                const ConvSrc &s = si ? p.src[1] : p.src[0];
                const int kind = c < p.Cin ? s.kind : SRC_NONE;
                const int cl = c - (si ? C0 : 0);
                const int sdt = s.sdt ? s.sdt - 1 : Store<DT>::v;
                const size_t cb = (size_t)s.coff + cl;
                const PixSrc *tabp = sm.ps[si];
                const ST *sp = (const ST *)s.ptr;
                constexpr int PSTEP = 256 / KCG;                // pixels between a thread's elements
                constexpr int NE = (NPIX + PSTEP - 1) / PSTEP;  // patch elements per thread
                constexpr int GR = 4;                           // resized elements (4 corners each) per step
                constexpr int NGR = (NE + GR - 1) / GR;
                constexpr int GT = NE < 8 ? NE : 8;             // plain elements per step
                constexpr int NGT = (NE + GT - 1) / GT;
                constexpr int NW = TAPS * TN * KCG;             // weight vectors of the chunk
                constexpr int EWT = (NW + 255) / 256;
                constexpr int GW = 8;
                constexpr int NGW = (EWT + GW - 1) / GW;
                constexpr int NG1 = NGR > NGT ? NGR : NGT;
                constexpr int NG = NG1 > NGW ? NG1 : NGW;
                const int pix0 = tid / KCG;
                // a chunk that holds only the two channels of the network input x0
                // (the first layer, and the last chunk of the layer before the final
                // one) is staged by all threads below, one patch pixel each
                const bool x0_only = c0 + GS >= p.Cin &&
                                     ((c0 == 0 && p.src[0].kind == SRC_X0) ||
                                      (c0 == C0 && p.src[1].kind == SRC_X0));
                // grouped fast paths for sources stored in the layer's storage dtype
                // (INT8 layers: BF16 maps, quantised while staging)
                const bool fast_resize = kind == SRC_RESIZE && sdt == SD && !x0_only;
                const bool fast_plain = (kind == SRC_TENSOR || kind == SRC_ZINS) && sdt == SD && !x0_only;
#pragma unroll
                for (int gi = 0; gi < NG; ++gi) {
                    // -- issue
                    SVec ra[GR][4];
                    PixSrc rq[GR];
                    bool rok[GR];
                    if (gi < NGR && fast_resize) {
#pragma unroll
                        for (int j = 0; j < GR; ++j) {
                            const int k = gi * GR + j;
                            const int pix = pix0 + k * PSTEP;
                            const bool in = k < NE && pix < NPIX;
                            rq[j] = tabp[in ? pix : 0];
                            rok[j] = in && rq[j].p[0] >= 0;
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                ra[j][r] = *(const SVec *)(sp + (size_t)(rok[j] ? rq[j].p[r] : 0) * s.pitch + cb);
                        }
                    }
                    SVec ta[GT];
                    bool tok[GT];
                    if (gi < NGT && fast_plain) {
#pragma unroll
                        for (int j = 0; j < GT; ++j) {
                            const int k = gi * GT + j;
                            const int pix = pix0 + k * PSTEP;
                            const bool in = k < NE && pix < NPIX;
                            const int pi = tabp[in ? pix : 0].p[0];
                            tok[j] = in && pi >= 0;
                            ta[j] = *(const SVec *)(sp + (size_t)(tok[j] ? pi : 0) * s.pitch + cb);
                        }
                    }
                    vec wv[GW];
                    bool wok[GW];
                    if (gi < NGW) {
#pragma unroll
                        for (int j = 0; j < GW; ++j) {
                            const int k = gi * GW + j;
                            const int e = k * 256 + tid;
                            const int wcg = e % KCG, r = e / KCG;
                            const int n = r % TN, tap = r / TN;
                            const int wc = c0 + wcg * GS, ng = n0 + n;
                            wok[j] = k < EWT && e < NW && ng < p.n_pad && wc < p.cin_pad;
                            wv[j] = *(const vec *)(wpk + (wok[j] ? ((size_t)tap * p.n_pad + ng) * p.cin_pad + wc : 0));
                        }
                    }
                    // -- commit to LDS
                    if (gi < NGR && fast_resize) {
#pragma unroll
                        for (int j = 0; j < GR; ++j) {
                            const int k = gi * GR + j;
                            const int pix = pix0 + k * PSTEP;
                            if (k >= NE || pix >= NPIX) continue;
                            float v[GS];
                            if constexpr (DT == SV_I8) {
                                // INT8 codes are defined on the separable FP32 expression
#pragma unroll
                                for (int i = 0; i < GS; ++i) {
                                    const float x00 = Elem<SD>::load((const ST *)&ra[j][0] + i);
                                    const float x01 = Elem<SD>::load((const ST *)&ra[j][1] + i);
                                    const float x10 = Elem<SD>::load((const ST *)&ra[j][2] + i);
                                    const float x11 = Elem<SD>::load((const ST *)&ra[j][3] + i);
                                    const float top = (1.f - rq[j].lx) * x00 + rq[j].lx * x01;
                                    const float bot = (1.f - rq[j].lx) * x10 + rq[j].lx * x11;
                                    v[i] = rok[j] ? (1.f - rq[j].ly) * top + rq[j].ly * bot : 0.f;
                                }
                            } else {
                                // the four corner weights once per pixel, then one
                                // multiply and three fused multiply-adds per channel
                                const float ly = rq[j].ly, lx = rq[j].lx;
                                const float wy0 = 1.f - ly;
                                const float w00 = wy0 * (1.f - lx), w01 = wy0 * lx;
                                const float w10 = ly * (1.f - lx), w11 = ly * lx;
#pragma unroll
                                for (int i = 0; i < GS; ++i) {
                                    const float x00 = Elem<SD>::load((const ST *)&ra[j][0] + i);
                                    const float x01 = Elem<SD>::load((const ST *)&ra[j][1] + i);
                                    const float x10 = Elem<SD>::load((const ST *)&ra[j][2] + i);
                                    const float x11 = Elem<SD>::load((const ST *)&ra[j][3] + i);
                                    const float r = fmaf(w11, x11, fmaf(w10, x10, fmaf(w01, x01, w00 * x00)));
                                    v[i] = rok[j] ? r : 0.f;
                                }
                            }
                            *(vec *)&patch[pix * KCP + cg * GS] = pack_vec<DT, GS>(v, qinv);
                        }
                    }
                    if (gi < NGT && fast_plain) {
#pragma unroll
                        for (int j = 0; j < GT; ++j) {
                            const int k = gi * GT + j;
                            const int pix = pix0 + k * PSTEP;
                            if (k >= NE || pix >= NPIX) continue;
                            if constexpr (SD != DT) {
                                float v[GS];
#pragma unroll
                                for (int i = 0; i < GS; ++i)
                                    v[i] = tok[j] ? Elem<SD>::load((const ST *)&ta[j] + i) : 0.f;
                                *(vec *)&patch[pix * KCP + cg * GS] = pack_vec<DT, GS>(v, qinv);
                            } else {
                                vec o = ta[j];
                                if (!tok[j]) {
#pragma unroll
                                    for (int i = 0; i < GS; ++i) o[i] = 0;
                                }
                                *(vec *)&patch[pix * KCP + cg * GS] = o;
                            }
                        }
                    }
                    if (gi < NGW) {
#pragma unroll
                        for (int j = 0; j < GW; ++j) {
                            const int k = gi * GW + j;
                            const int e = k * 256 + tid;
                            if (k >= EWT || e >= NW) continue;
                            const int wcg = e % KCG, r = e / KCG;
                            const int n = r % TN, tap = r / TN;
                            vec o = wv[j];
                            if (!wok[j]) {
#pragma unroll
                                for (int i = 0; i < GS; ++i) o[i] = 0;
                            }
                            *(vec *)&wl[(tap * TN + n) * KCP + wcg * GS] = o;
                        }
                    }
                }
                // -- the remaining kinds, element by element: a source stored in
                // another dtype or the network input x0 (groups past Cin are
                // never read by the MFMA steps and are not written)
                if (x0_only) {
                    const ConvSrc &sx = c0 == 0 ? p.src[0] : p.src[1];
                    const PixSrc *tx = sm.ps[c0 == 0 ? 0 : 1];
                    constexpr int NX = (NPIX + 255) / 256;
                    uint32_t dv[NX], iv[NX];
                    bool okx[NX];
#pragma unroll
                    for (int k = 0; k < NX; ++k) {  // all loads first
                        const int pix = tid + k * 256;
                        const int pi = pix < NPIX ? tx[pix].p[0] : -1;
                        okx[k] = pi >= 0;
                        dv[k] = ((const uint8_t *)sx.ptr)[okx[k] ? pi : 0];
                        iv[k] = sx.img[okx[k] ? pi : 0];
                    }
#pragma unroll
                    for (int k = 0; k < NX; ++k) {
                        const int pix = tid + k * 256;
                        if (pix >= NPIX) continue;
                        float v[GS];
#pragma unroll
                        for (int i = 0; i < GS; ++i) v[i] = 0.f;
                        if (okx[k]) {
                            v[0] = sx.scale0 * (float)dv[k];
                            v[1] = (float)iv[k] * (1.0f / 256.0f);
                        }
                        *(vec *)&patch[pix * KCP] = pack_vec<DT, GS>(v, qinv);
                    }
                }
                if (kind == SRC_NONE && c < c0 + nsub * KCB) {
                    // a channel group past Cin (or past the range) that the MFMA
                    // steps read: zeros (stale LDS could hold NaN, and NaN x 0 is NaN)
                    vec z;
#pragma unroll
                    for (int i = 0; i < GS; ++i) z[i] = 0;
#pragma unroll
                    for (int k = 0; k < NE; ++k) {
                        const int pix = pix0 + k * PSTEP;
                        if (pix < NPIX) *(vec *)&patch[pix * KCP + cg * GS] = z;
                    }
                } else if (!x0_only && !fast_resize && !fast_plain && kind != SRC_NONE) {
#pragma unroll
                    for (int k = 0; k < NE; ++k) {
                        const int pix = pix0 + k * PSTEP;
                        if (pix >= NPIX) continue;
                        float v[GS];
#pragma unroll
                        for (int i = 0; i < GS; ++i) v[i] = 0.f;
                        const PixSrc q = tabp[pix];
                        if (q.p[0] >= 0) {
                            if (kind == SRC_RESIZE) {
                                float a4[4][GS];
#pragma unroll
                                for (int r = 0; r < 4; ++r)
                                    load_px<DT, GS>(s.ptr, (size_t)q.p[r] * s.pitch + cb, sdt, a4[r]);
#pragma unroll
                                for (int i = 0; i < GS; ++i) {
                                    const float top = (1.f - q.lx) * a4[0][i] + q.lx * a4[1][i];
                                    const float bot = (1.f - q.lx) * a4[2][i] + q.lx * a4[3][i];
                                    v[i] = (1.f - q.ly) * top + q.ly * bot;
                                }
                            } else if (kind == SRC_TENSOR || kind == SRC_ZINS) {
                                load_px<DT, GS>(s.ptr, (size_t)q.p[0] * s.pitch + cb, sdt, v);
                            } else if (kind == SRC_X0) {
                                v[0] = s.scale0 * (float)((const uint8_t *)s.ptr)[q.p[0]];
                                v[1] = (float)s.img[q.p[0]] * (1.0f / 256.0f);
                            }
                        }
                        *(vec *)&patch[pix * KCP + cg * GS] = pack_vec<DT, GS>(v, qinv);
                    }
                }
            }
            __syncthreads();
            // ---- MFMA, base chunk by base chunk, tap by tap ---------------------
            // Step = tap; lane group g supplies channel group g of the chunk
            // (channels past Cin are zero in the patch and the weights), so each
            // operand address is a per-lane base plus a compile-time offset.  The
            // chunk loop stays rolled: one set of accumulator registers carried
            // through it, no copies between branches.
#pragma clang loop unroll(disable)
            for (int sub = 0; sub < nsub; ++sub) {
                const T *pb = patch + (size_t)((wm * MBW) * S * PW + r16 * S) * KCP + (sub * KCGB + g) * GS;
                const T *pa = wl + (size_t)((wn * NBW) * 16 + r16) * KCP + (sub * KCGB + g) * GS;
#pragma unroll
                for (int tap = 0; tap < TAPS; ++tap) {
                    const int u = tap / KS, v = tap % KS;
                    vec bf[MBW], af[NBW];
#pragma unroll
                    for (int mb = 0; mb < MBW; ++mb)
                        bf[mb] = *(const vec *)(pb + ((mb * S + u) * PW + v) * KCP);
#pragma unroll
                    for (int nb = 0; nb < NBW; ++nb)
                        af[nb] = *(const vec *)(pa + (tap * TN + nb * 16) * KCP);
#pragma unroll
                    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
                        for (int nb = 0; nb < NBW; ++nb) acc[mb][nb] = M::run(af[nb], bf[mb], acc[mb][nb]);
                }
            }
        }

        if (c_x0 < c_end) x0_packed(p, sm, acc, qinv, n0, wm, wn, g, r16);

        // ---- epilogue -------------------------------------------------------
        if constexpr (WN == 1) {
            if (p.proj_out) {  // launches set it only for tiles that hold every channel
                project_epilogue(p, G, acc, bpre, spre);
                return;
            }
        }
        // the FP32 partial of this channel range, or bias, activation,
        // backward terms and the NHWC store
        float lmax = 0.f;
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb) {
            const int oy = oy0 + wm * MBW + mb, ox = ox0 + r16;
            if (oy >= G.Ho || ox >= G.Wo) continue;
            size_t pix = (size_t)(G.obase + (long long)oy * G.Wo + ox);
            if (p.ophase) {  // one parity class of an interleaved output
                const int py = (p.ophase - 1) >> 1, px = (p.ophase - 1) & 1;
                pix = ((size_t)G.b * p.Ho_full + 2 * oy + py) * p.Wo_full + 2 * ox + px;
            }
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
                const int nbase = n0 + (wn * NBW + nb) * 16 + 4 * g;
                f32x4 av;
                if constexpr (DT == SV_I8) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) av[i] = (float)acc[mb][nb][i] * spre[nb][i];
                } else {
                    av = acc[mb][nb];
                }
                if (p.ksplit > 1) {
                    // n_pad is a multiple of 16: the four channels are all in or all out
                    // (INT8 layers never split)
                    if (nbase < p.n_pad)
                        *(f32x4 *)&p.part[((size_t)kz * p.B * G.Ho * G.Wo + pix) * p.n_pad + nbase] = av;
                } else {
                    const float r[4] = {av[0], av[1], av[2], av[3]};
                    lmax = fmaxf(lmax, conv_epilogue<DT>(p, pix, nbase, r, bpre[nb]));
                }
            }
        }
        if (p.amax_out && p.ksplit <= 1)
            record_amax_wg(p, lmax, (int)(blockIdx.x * 7u + blockIdx.y * 13u + blockIdx.z), sm.red);
    }
};

// Uniform batch: one workgroup per (column tile, row tile, image x channel tile).
template <int DT, int KS, int S, int TH, int TN, int WM, int KCM>
__device__ __forceinline__ void conv_uniform(const ConvParams &p,
                                             typename ConvTile<DT, KS, S, TH, TN, WM, KCM>::Smem &sm)
{
    using CT = ConvTile<DT, KS, S, TH, TN, WM, KCM>;
    const int ntn = (p.Cout + TN - 1) / TN;
    const int ksplit = p.ksplit > 1 ? p.ksplit : 1;
    // XCD-aware order: workgroups go round robin to the eight XCDs (each with
    // its own L2), so hardware id i is given logical tile (i % 8) * q + i / 8,
    // q = N / 8 (a transpose; the last N % 8 ids keep their own): each XCD then
    // works on one contiguous run of the (image, channel tile, split, row,
    // column) order and fetches only the weights and inputs of that run
    const int gx = (int)gridDim.x, gy = (int)gridDim.y;
    const int nblk = gx * gy * (int)gridDim.z;
    const int hw = (int)blockIdx.x + gx * ((int)blockIdx.y + gy * (int)blockIdx.z);
    const int q8 = nblk / 8;
    const int lid = hw < 8 * q8 ? (hw % 8) * q8 + hw / 8 : hw;
    const int bz = lid / (gx * gy), rem = lid - bz * (gx * gy);
    const int by = rem / gx, bx = rem - by * gx;
    const int kz = bz % ksplit, zz = bz / ksplit;
    const int b = zz / ntn;
    ConvGeo G;
    G.Hi = p.Hi; G.Wi = p.Wi; G.Ho = p.Ho; G.Wo = p.Wo;
    for (int i = 0; i < 2; ++i) {
        G.hs[i] = p.src[i].hs;
        G.ws[i] = p.src[i].ws;
        G.sbase[i] = (long long)b * p.src[i].hs * p.src[i].ws;
    }
    G.obase = (long long)b * p.Ho * p.Wo;
    G.b = b;
    G.n0 = (zz % ntn) * TN;
    G.oy0 = by * TH;
    G.ox0 = bx * CT::TW;
    CT::run(p, G, sm, kz);
}

template <int DT, int KS, int S, int TH, int TN, int WM, int KCM>
__global__ void __launch_bounds__(256) k_conv(const ConvParams p)
{
    __shared__ __attribute__((aligned(16))) typename ConvTile<DT, KS, S, TH, TN, WM, KCM>::Smem sm;
    conv_uniform<DT, KS, S, TH, TN, WM, KCM>(p, sm);
}

// The same, its registers held to two waves per SIMD (256 VGPRs, AGPRs
// included), for the INT8 16-row stride-1 tiles, which the compiler would otherwise
// take a few registers past that (one wave per SIMD, half the workgroups).
template <int DT, int KS, int S, int TH, int TN, int WM, int KCM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_conv_w2(const ConvParams p)
{
    __shared__ __attribute__((aligned(16))) typename ConvTile<DT, KS, S, TH, TN, WM, KCM>::Smem sm;
    conv_uniform<DT, KS, S, TH, TN, WM, KCM>(p, sm);
}

// Pair table: persistent loop over the stage's tiles of every pair.  It
// forms the pixel table directly (no separable form): the separable form's
// registers would take some of these kernels past 256 VGPRs (AGPRs
// included), one wave per SIMD instead of two.
template <int DT, int KS, int S, int TH, int TN, int WM, int KCM>
__global__ void __launch_bounds__(256) k_conv_tab(const ConvParams p)
{
    using CT = ConvTile<DT, KS, S, TH, TN, WM, KCM>;
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
        G.b = 0;
        const int local = t - cum[i];
        const int tx = cdiv_d(G.Wo, CT::TW), ty = cdiv_d(G.Ho, TH);
        const int nt = local / (tx * ty), r = local - nt * tx * ty;
        G.n0 = nt * TN;
        G.oy0 = (r / tx) * TH;
        G.ox0 = (r % tx) * CT::TW;
        CT::template run<false>(p, G, sm, 0);
        (void)ntn;
    }
}

// Second pass of a split reduction: adds the ksplit FP32 partials of four
// channels of one pixel in range order, then applies the epilogue.  Every
// partial and the bias are loaded before the first addition (the ranges that
// do not exist read range 0 and are not added), so one memory latency is
// paid per element instead of one per range.
template <int DT>
__global__ void __launch_bounds__(256) k_conv_split_reduce(const ConvParams p, int npix)
{
    const int ng = p.n_pad / 4;
    const size_t total = (size_t)npix * ng;
    float lmax = 0.f;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t pix = e / ng;
        const int nbase = (int)(e - pix * ng) * 4;
        if (nbase >= p.Cout) continue;
        float b[4];
        conv_bias4<DT>(p, nbase, b);
        f32x4 q[CONV_MAX_SPLIT];
#pragma unroll
        for (int z = 0; z < CONV_MAX_SPLIT; ++z) {
            const size_t zz = z < p.ksplit ? (size_t)z : 0;
            q[z] = *(const f32x4 *)&p.part[(zz * npix + pix) * p.n_pad + nbase];
        }
        f32x4 s = q[0];
#pragma unroll
        for (int z = 1; z < CONV_MAX_SPLIT; ++z) {
            if (z < p.ksplit) {
                s[0] += q[z][0]; s[1] += q[z][1]; s[2] += q[z][2]; s[3] += q[z][3];
            }
        }
        const float r[4] = {s[0], s[1], s[2], s[3]};
        lmax = fmaxf(lmax, conv_epilogue<DT>(p, pix, nbase, r, b));
    }
    if (p.amax_out) record_amax(p, lmax, (int)blockIdx.x);
}

// The second pass of a split reduction over the B Ho Wo output pixels of p.
template <int DT>
static sv_status launch_reduce(const ConvParams &p, hipStream_t st) {
    const int npix = p.B * p.Ho * p.Wo;
    const long long work = (long long)npix * (p.n_pad / 4);
    const int blocks = (int)std::min<long long>((work + 255) / 256, 4096);
    hipLaunchKernelGGL(k_conv_split_reduce<DT>, dim3(blocks), dim3(256), 0, st, p, npix);
    SV_LAUNCH_CHECK("k_conv_split_reduce");
    return SV_OK;
}

// grid <= 0: uniform launch (split over p.ksplit channel ranges when p.ksplit > 1);
// grid > 0: persistent launch over p.tab.
template <int DT, int KS, int S, int TH, int TN, int WM, int KCM>
static sv_status launch_one(const ConvParams &p, int pgrid, hipStream_t st) {
    if constexpr (!ConvTile<DT, KS, S, TH, TN, WM, KCM>::FITS) {
        return SV_ERR_UNSUPPORTED;
    } else {
    if (pgrid > 0) {
        const long long g = resident_grid((const void *)k_conv_tab<DT, KS, S, TH, TN, WM, KCM>, 0, pgrid);
        hipLaunchKernelGGL((k_conv_tab<DT, KS, S, TH, TN, WM, KCM>), dim3((unsigned)g), dim3(256), 0, st, p);
        SV_LAUNCH_CHECK("k_conv_tab");
        return SV_OK;
    }
    const int ksplit = p.ksplit > 1 ? p.ksplit : 1;
    const long long gz = (long long)p.B * cdiv(p.Cout, TN) * ksplit;
    if (gz > 65535) return SV_ERR_SHAPE;
    dim3 grid(cdiv(p.Wo, 16), cdiv(p.Ho, TH), (unsigned)gz);
    if constexpr (DT == SV_I8 && TH == 16 && S == 1)
        hipLaunchKernelGGL((k_conv_w2<DT, KS, S, TH, TN, WM, KCM>), grid, dim3(256), 0, st, p);
    else
        hipLaunchKernelGGL((k_conv<DT, KS, S, TH, TN, WM, KCM>), grid, dim3(256), 0, st, p);
    SV_LAUNCH_CHECK("k_conv");
    if (ksplit > 1 && !p.defer_sum) return launch_reduce<DT>(p, st);
    return SV_OK;
    }
}

template <int DT, int KS, int S>
static sv_status launch_cfg(int cfg, const ConvParams &p, int pg, hipStream_t st) {
    switch (cfg) {
#define SV_CFG(i, TH, TN, WM, KCM, name) \
    case i: return launch_one<DT, KS, S, TH, TN, WM, KCM>(p, pg, st);
        SV_CONV_CFGS(SV_CFG)
#undef SV_CFG
    default: return SV_ERR_RANGE;
    }
}

template <int DT, int KS, int S>
static bool fits_cfg(int cfg) {
    switch (cfg) {
#define SV_CFG(i, TH, TN, WM, KCM, name) \
    case i: return ConvTile<DT, KS, S, TH, TN, WM, KCM>::FITS;
        SV_CONV_CFGS(SV_CFG)
#undef SV_CFG
    default: return false;
    }
}

// Whether tile shape `cfg` fits the LDS for this kernel size and stride.
template <int DT>
static bool fits_dt(int ks, int stride, int cfg) {
    if (ks == 3 && stride == 1) return fits_cfg<DT, 3, 1>(cfg);
    if (ks == 3 && stride == 2) return fits_cfg<DT, 3, 2>(cfg);
    if (ks == 1 && stride == 1) return fits_cfg<DT, 1, 1>(cfg);
    return false;
}

// 5x5 kernels (the Table I network), one stride per instantiation file
template <int DT, int S>
static sv_status launch_dt5(int cfg, const ConvParams &p, int pg, hipStream_t st) {
    return launch_cfg<DT, 5, S>(cfg, p, pg, st);
}
template <int DT, int S>
static bool fits_dt5(int cfg) { return fits_cfg<DT, 5, S>(cfg); }

template <int DT>
static sv_status launch_dt(int ks, int stride, int cfg, const ConvParams &p, int pg, hipStream_t st) {
    if (ks == 3 && stride == 1) return launch_cfg<DT, 3, 1>(cfg, p, pg, st);
    if (ks == 3 && stride == 2) return launch_cfg<DT, 3, 2>(cfg, p, pg, st);
    if (ks == 1 && stride == 1) return launch_cfg<DT, 1, 1>(cfg, p, pg, st);
    return SV_ERR_UNSUPPORTED;
}


}  // namespace sv
