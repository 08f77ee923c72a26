// Backward pass of the refinement network: the exact adjoint of the forward
// pass, for  loss = sum(dout * out) + kl_weight * KL  (Sec. III-B2 in the
// reading documented in sv.h).
//
//   * input gradients (dgrad) reuse the forward implicit-GEMM kernel with the
//     adjoint weight pack (rows = the layer's inputs, kernel flipped); the
//     stride-2 encoder layers see the output gradient with zeros inserted
//     (SRC_ZINS), and the epilogue adds the skip-connection gradient and
//     multiplies by the leaky-ReLU derivative of the layer below;
//   * weight gradients (wgrad) are an MFMA GEMM reducing over pixels: every
//     workgroup owns a fixed slice of output tiles and writes its partial sums;
//     a second kernel adds the partials in a fixed order (no float atomics), so
//     gradients are bitwise reproducible;
//   * the bilinear resizes' adjoints are gathers (each coarse pixel collects
//     from the fine pixels whose interpolation reads it), fused with the
//     leaky-ReLU derivative;
//   * the final layer's adjoint is one gather kernel producing the per-tap
//     projection gradient and, through the 9 x (c1+2) weights, the gradient of
//     G0's pre-activation;
//   * the encoder activations are recomputed from x0 (checkpointing).
#include "mfma.h"
#include "net.h"
#include "prof.h"

namespace sv {

// One element of a map stored in dtype sdt, as FP32.
__device__ __forceinline__ float ld_el(const void *p, size_t i, int sdt) {
    if (sdt == SV_F32) return ((const float *)p)[i];
    const uint16_t h = ((const uint16_t *)p)[i];
    return sdt == SV_BF16 ? bf16_bits_to_f32(h) : f16_bits_to_f32(h);
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[o][tap][c] = sum over output pixels m of
//   dY[m][o] * X[m shifted by tap][c],  db[o] = sum_m dY[m][o].
// Workgroup (split, channel chunk, output chunk); tiles of 4 x 16 output
// pixels, visited in a fixed order per split.  The X patch is staged as in the
// forward pass, then unfolded in LDS into [tap][c][m] so that both MFMA
// operands read 8 (BF16) or 4 (FP32) consecutive pixels per lane.
// ---------------------------------------------------------------------------
struct WgradParams {
    ConvSrc src[2];
    int B, Hi, Wi, Ho, Wo, Cin, Cout;
    const float *dy;
    int dy_pitch;
    float *part;    // [split][o_pad][taps][cinp]
    float *part_b;  // [split][o_pad]
    int o_pad, cinp;
    int ntiles, tiles_x, tiles_y;
};

constexpr int WG_TH = 4, WG_TW = 16, WG_MT = WG_TH * WG_TW, WG_OC = 32;
static inline int wg_kcw(int ks) { return ks == 1 ? 64 : 16; }

template <int DT, int KS, int S>
__global__ void __launch_bounds__(256) k_wgrad(const WgradParams p)
{
    using M = Mfma<DT>;
    using T = typename M::T;
    using vec = typename M::vec;
    constexpr int GS = M::GS;
    constexpr int TAPS = KS * KS, PAD = (KS - 1) / 2;
    constexpr int KCW = KS == 1 ? 64 : 16;
    constexpr int PH = (WG_TH - 1) * S + KS, PW = (WG_TW - 1) * S + KS;
    constexpr int MTP = WG_MT + GS;        // padded pixel rows
    constexpr int KCP = KCW + GS;          // padded channel rows of the patch
    constexpr int KB = TAPS * KCW / 16;    // column blocks
    constexpr int NB = (WG_OC / 16) * KB;  // output blocks of the workgroup
    constexpr int NBW = (NB + 3) / 4;      // per wave
    constexpr int MK = 4 * GS;             // pixels per MFMA step

    __shared__ __attribute__((aligned(16))) T dyT[WG_OC * MTP];
    __shared__ __attribute__((aligned(16))) T xp[PH * PW * KCP];
    __shared__ __attribute__((aligned(16))) T xcol[TAPS * KCW * MTP];
    __shared__ float bsum[256];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int split = blockIdx.x, c0 = blockIdx.y * KCW, o0 = blockIdx.z * WG_OC;
    const bool do_bias = blockIdx.y == 0;

    f32x4 acc[NBW];
#pragma unroll
    for (int j = 0; j < NBW; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float sb = 0.f;

    for (int tile = split; tile < p.ntiles; tile += gridDim.x) {
        const int per_img = p.tiles_x * p.tiles_y;
        const int b = tile / per_img, rem = tile - b * per_img;
        const int oy0 = (rem / p.tiles_x) * WG_TH, ox0 = (rem % p.tiles_x) * WG_TW;
        const int iy0 = oy0 * S - PAD, ix0 = ox0 * S - PAD;
        __syncthreads();
        // output gradient tile, transposed to [o][m]
        for (int e = tid; e < WG_OC * WG_MT; e += 256) {
            const int o = e % WG_OC, m = e / WG_OC;
            const int oy = oy0 + m / WG_TW, ox = ox0 + m % WG_TW;
            float v = 0.f;
            if (oy < p.Ho && ox < p.Wo && o0 + o < p.Cout)
                v = p.dy[(((size_t)b * p.Ho + oy) * p.Wo + ox) * p.dy_pitch + o0 + o];
            sb += v;  // thread tid always sees o = tid % 32
            dyT[o * MTP + m] = Elem<DT>::make(v);
        }
        // input patch (zero padded), NHWC in LDS
        for (int e = tid; e < PH * PW * (KCW / GS); e += 256) {
            const int cg = e % (KCW / GS), pix = e / (KCW / GS);
            const int py = pix / PW, px = pix - py * PW;
            const int yi = iy0 + py, xi = ix0 + px, c = c0 + cg * GS;
            float v[GS];
#pragma unroll
            for (int i = 0; i < GS; ++i) v[i] = 0.f;
            if (yi >= 0 && yi < p.Hi && xi >= 0 && xi < p.Wi && c < p.Cin) {
                const int si = c < p.src[0].C ? 0 : 1;
                const ConvSrc &s = p.src[si];
                const int cl = c - (si ? p.src[0].C : 0);
                const int sdt = s.sdt ? s.sdt - 1 : DT;
                if (s.kind == SRC_TENSOR) {
                    const size_t off = (((size_t)b * s.hs + yi) * s.ws + xi) * s.pitch + s.coff + cl;
#pragma unroll
                    for (int i = 0; i < GS; ++i) v[i] = ld_el(s.ptr, off + i, sdt);
                } else if (s.kind == SRC_ZINS) {
                    // zeros between samples: only even positions hold the map
                    if (((yi | xi) & 1) == 0) {
                        const size_t off = (((size_t)b * s.hs + (yi >> 1)) * s.ws + (xi >> 1)) * s.pitch + s.coff + cl;
#pragma unroll
                        for (int i = 0; i < GS; ++i) v[i] = ld_el(s.ptr, off + i, sdt);
                    }
                } else if (s.kind == SRC_RESIZE) {
                    int y0, y1, x0, x1;
                    float ly, lx;
                    bilin(yi, s.hs, p.Hi, y0, y1, ly);
                    bilin(xi, s.ws, p.Wi, x0, x1, lx);
                    const size_t rb = (size_t)b * s.hs, cb = (size_t)s.coff + cl;
                    const size_t o00 = ((rb + y0) * s.ws + x0) * s.pitch + cb;
                    const size_t o01 = ((rb + y0) * s.ws + x1) * s.pitch + cb;
                    const size_t o10 = ((rb + y1) * s.ws + x0) * s.pitch + cb;
                    const size_t o11 = ((rb + y1) * s.ws + x1) * s.pitch + cb;
#pragma unroll
                    for (int i = 0; i < GS; ++i) {
                        const float top = (1.f - lx) * ld_el(s.ptr, o00 + i, sdt) + lx * ld_el(s.ptr, o01 + i, sdt);
                        const float bot = (1.f - lx) * ld_el(s.ptr, o10 + i, sdt) + lx * ld_el(s.ptr, o11 + i, sdt);
                        v[i] = (1.f - ly) * top + ly * bot;
                    }
                } else if (s.kind == SRC_X0) {
                    const size_t o = ((size_t)b * s.hs + yi) * s.ws + xi;
                    v[0] = s.scale0 * (float)((const uint8_t *)s.ptr)[o];
                    v[1] = (float)s.img[o] * (1.0f / 256.0f);
                }
            }
#pragma unroll
            for (int i = 0; i < GS; ++i) xp[(py * PW + px) * KCP + cg * GS + i] = Elem<DT>::make(v[i]);
        }
        __syncthreads();
        // unfold: xcol[tap * KCW + c][m]
        for (int e = tid; e < TAPS * KCW * WG_MT; e += 256) {
            const int m = e % WG_MT, kc = e / WG_MT;
            const int c = kc % KCW, tap = kc / KCW;
            const int u = tap / KS, v = tap % KS;
            const int ty = m / WG_TW, tx = m % WG_TW;
            xcol[kc * MTP + m] = xp[((ty * S + u) * PW + tx * S + v) * KCP + c];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NBW; ++j) {
            const int bi = wave + 4 * j;
            if (bi < NB) {
                const int ob = bi / KB, kb = bi % KB;
#pragma unroll
                for (int ms = 0; ms < WG_MT; ms += MK) {
                    const vec a = *(const vec *)&dyT[(ob * 16 + r16) * MTP + ms + GS * g];
                    const vec bb = *(const vec *)&xcol[(kb * 16 + r16) * MTP + ms + GS * g];
                    acc[j] = M::run(a, bb, acc[j]);
                }
            }
        }
    }
    // partials: lane holds D[o = ob*16 + 4g + r][col = kb*16 + r16]
#pragma unroll
    for (int j = 0; j < NBW; ++j) {
        const int bi = wave + 4 * j;
        if (bi >= NB) continue;
        const int ob = bi / KB, kb = bi % KB;
        const int col = kb * 16 + r16, tap = col / KCW, c = c0 + col % KCW;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = o0 + ob * 16 + 4 * g + r;
            p.part[(((size_t)split * p.o_pad + o) * TAPS + tap) * p.cinp + c] = acc[j][r];
        }
    }
    if (do_bias) {
        bsum[tid] = sb;
        __syncthreads();
        if (tid < WG_OC) {
            float t = 0.f;
            for (int k = 0; k < 256 / WG_OC; ++k) t += bsum[tid + k * WG_OC];
            p.part_b[(size_t)split * p.o_pad + o0 + tid] = t;
        }
    }
}

// Adds the partials of all splits in split order and writes the canonical
// (OIHW, then bias) gradient of one layer.  final_layer: the "outputs" are
// the 9 taps of the single-output final layer: dW[0][c][tap].
__global__ void k_wgrad_reduce(const float *__restrict__ part, const float *__restrict__ part_b,
                               int splits, int o_pad, int taps, int cinp, int Cout, int Cin,
                               int final_layer, float *__restrict__ grad)
{
    const int nw = Cout * Cin * taps;
    const int n = nw + (final_layer ? 0 : Cout);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        float s = 0.f;
        if (e < nw) {
            int o, c, tap;
            if (final_layer) {  // canonical index c * 9 + tap, "output" o = tap
                c = e / Cout;
                o = e % Cout;
                tap = 0;
            } else {
                o = e / (Cin * taps);
                c = (e / taps) % Cin;
                tap = e % taps;
            }
            for (int k = 0; k < splits; ++k) s += part[(((size_t)k * o_pad + o) * taps + tap) * cinp + c];
        } else {
            const int o = e - nw;
            for (int k = 0; k < splits; ++k) s += part_b[(size_t)k * o_pad + o];
        }
        grad[e] = s;
    }
}

struct WgradPlan { int splits, o_pad, cinp, taps, ntiles, tx, ty, nc, no; };

static WgradPlan wgrad_plan(int B, int Ho, int Wo, int Cin, int Cout, int ks) {
    WgradPlan w;
    const int kcw = wg_kcw(ks);
    w.taps = ks * ks;
    w.o_pad = (Cout + WG_OC - 1) / WG_OC * WG_OC;
    w.cinp = (Cin + kcw - 1) / kcw * kcw;
    w.tx = cdiv(Wo, WG_TW);
    w.ty = cdiv(Ho, WG_TH);
    w.ntiles = B * w.tx * w.ty;
    w.nc = w.cinp / kcw;
    w.no = w.o_pad / WG_OC;
    const int groups = w.nc * w.no;
    int sp = 1024 / groups;
    if (sp < 1) sp = 1;
    if (sp > w.ntiles) sp = w.ntiles;
    w.splits = sp;
    return w;
}

static size_t wgrad_part_floats(const WgradPlan &w) {
    return (size_t)w.splits * w.o_pad * w.taps * w.cinp + (size_t)w.splits * w.o_pad;
}

template <int DT>
static sv_status launch_wgrad_dt(int ks, int stride, const WgradParams &p, const WgradPlan &w,
                                 hipStream_t st) {
    dim3 grid(w.splits, w.nc, w.no);
    if (ks == 3 && stride == 1)
        hipLaunchKernelGGL((k_wgrad<DT, 3, 1>), grid, dim3(256), 0, st, p);
    else if (ks == 3 && stride == 2)
        hipLaunchKernelGGL((k_wgrad<DT, 3, 2>), grid, dim3(256), 0, st, p);
    else if (ks == 1 && stride == 1)
        hipLaunchKernelGGL((k_wgrad<DT, 1, 1>), grid, dim3(256), 0, st, p);
    else if (ks == 5 && stride == 1)
        hipLaunchKernelGGL((k_wgrad<DT, 5, 1>), grid, dim3(256), 0, st, p);
    else if (ks == 5 && stride == 2)
        hipLaunchKernelGGL((k_wgrad<DT, 5, 2>), grid, dim3(256), 0, st, p);
    else
        return SV_ERR_UNSUPPORTED;
    SV_LAUNCH_CHECK("k_wgrad");
    return SV_OK;
}

// One layer's weight and bias gradient into grad (its canonical slice).
static sv_status wgrad_layer(int dtype, int ks, int stride, ConvSrc s0, ConvSrc s1, int B, int Hi,
                             int Wi, int Ho, int Wo, int Cout, const float *dy, int dy_pitch,
                             float *part, int final_layer, float *grad, hipStream_t st) {
    const int Cin = s0.C + (s1.kind ? s1.C : 0);
    const WgradPlan w = wgrad_plan(B, Ho, Wo, Cin, Cout, ks);
    WgradParams p{};
    p.src[0] = s0; p.src[1] = s1;
    p.B = B; p.Hi = Hi; p.Wi = Wi; p.Ho = Ho; p.Wo = Wo; p.Cin = Cin; p.Cout = Cout;
    p.dy = dy; p.dy_pitch = dy_pitch;
    p.part = part;
    p.part_b = part + (size_t)w.splits * w.o_pad * w.taps * w.cinp;
    p.o_pad = w.o_pad; p.cinp = w.cinp;
    p.ntiles = w.ntiles; p.tiles_x = w.tx; p.tiles_y = w.ty;
    sv_status r;
    switch (dtype) {
    case SV_F32: r = launch_wgrad_dt<SV_F32>(ks, stride, p, w, st); break;
    case SV_BF16: r = launch_wgrad_dt<SV_BF16>(ks, stride, p, w, st); break;
    case SV_F16: r = launch_wgrad_dt<SV_F16>(ks, stride, p, w, st); break;
    default: return SV_ERR_DTYPE;
    }
    if (r != SV_OK) return r;
    const int n = Cout * Cin * w.taps + Cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(cdiv(n, 256)), dim3(256), 0, st, p.part, p.part_b,
                       w.splits, w.o_pad, w.taps, w.cinp, Cout, Cin, final_layer, grad);
    SV_LAUNCH_CHECK("k_wgrad_reduce");
    return SV_OK;
}

// The partial sums of one layer's weight and bias gradient (no reduction):
// part[split][o_pad][taps][cinp], then part_b[split][o_pad]; the shape of that
// layout is returned in `shape`.
size_t wgrad_partial_floats(int B, int Ho, int Wo, int Cin, int Cout, int ks) {
    return wgrad_part_floats(wgrad_plan(B, Ho, Wo, Cin, Cout, ks));
}

sv_status launch_wgrad_partials(int dtype, int ks, int stride, ConvSrc s0, ConvSrc s1, int B, int Hi, int Wi,
                                int Ho, int Wo, int Cout, const float *dy, int dy_pitch, float *part,
                                WgradShape &shape, hipStream_t st) {
    const int Cin = s0.C + (s1.kind ? s1.C : 0);
    const WgradPlan w = wgrad_plan(B, Ho, Wo, Cin, Cout, ks);
    WgradParams p{};
    p.src[0] = s0; p.src[1] = s1;
    p.B = B; p.Hi = Hi; p.Wi = Wi; p.Ho = Ho; p.Wo = Wo; p.Cin = Cin; p.Cout = Cout;
    p.dy = dy; p.dy_pitch = dy_pitch;
    p.part = part;
    p.part_b = part + (size_t)w.splits * w.o_pad * w.taps * w.cinp;
    p.o_pad = w.o_pad; p.cinp = w.cinp;
    p.ntiles = w.ntiles; p.tiles_x = w.tx; p.tiles_y = w.ty;
    shape.splits = w.splits; shape.o_pad = w.o_pad; shape.taps = w.taps; shape.cinp = w.cinp;
    switch (dtype) {
    case SV_F32: return launch_wgrad_dt<SV_F32>(ks, stride, p, w, st);
    case SV_BF16: return launch_wgrad_dt<SV_BF16>(ks, stride, p, w, st);
    case SV_F16: return launch_wgrad_dt<SV_F16>(ks, stride, p, w, st);
    default: return SV_ERR_DTYPE;
    }
}

// ---------------------------------------------------------------------------
// Bilinear resize adjoint (gather form) times the leaky-ReLU derivative of the
// coarse map:  out[b][i][j][c] = lrelu'(mask[b][i][j][c]) *
//   sum over fine (Y, X) of wy(Y -> i) wx(X -> j) in[b][Y][X][coff + c].
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bilin_weight_to(int o, int n_in, int n_out, int i) {
    int i0, i1;
    float lam;
    bilin(o, n_in, n_out, i0, i1, lam);
    return (i0 == i ? 1.f - lam : 0.f) + (i1 == i ? lam : 0.f);
}

template <int DT>
__global__ void k_resize_adj(const float *__restrict__ in, int ipitch, int icoff, int Hf, int Wf,
                             int Hc, int Wc, int C, const void *__restrict__ mask,
                             float *__restrict__ out, int B)
{
    const int cg4 = C / 4;
    const size_t n = (size_t)B * Hc * Wc * cg4;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const int cg = (int)(e % cg4);
        const size_t pix = e / cg4;
        const int j = (int)(pix % Wc), i = (int)((pix / Wc) % Hc), b = (int)(pix / ((size_t)Wc * Hc));
        const int ylo = max(0, ((i - 1) * Hf) / Hc - 1), yhi = min(Hf - 1, ((i + 2) * Hf) / Hc + 1);
        const int xlo = max(0, ((j - 1) * Wf) / Wc - 1), xhi = min(Wf - 1, ((j + 2) * Wf) / Wc + 1);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int Y = ylo; Y <= yhi; ++Y) {
            const float wy = bilin_weight_to(Y, Hc, Hf, i);
            if (wy == 0.f) continue;
            for (int X = xlo; X <= xhi; ++X) {
                const float wx = bilin_weight_to(X, Wc, Wf, j);
                if (wx == 0.f) continue;
                const float wgt = wy * wx;
                const f32x4 v = *(const f32x4 *)(in + (((size_t)b * Hf + Y) * Wf + X) * ipitch + icoff + 4 * cg);
                acc += wgt * v;
            }
        }
        const typename Elem<DT>::T *mk = (const typename Elem<DT>::T *)mask + pix * C + 4 * cg;
        f32x4 r;
        for (int k = 0; k < 4; ++k) r[k] = acc[k] * (Elem<DT>::load(mk + k) > 0.f ? 1.f : 0.1f);
        *(f32x4 *)(out + pix * C + 4 * cg) = r;
    }
}

static sv_status launch_resize_adj(int dtype, const float *in, int ipitch, int icoff, int Hf, int Wf,
                                   int Hc, int Wc, int C, const void *mask, float *out, int B,
                                   hipStream_t st) {
    const size_t n = (size_t)B * Hc * Wc * (C / 4);
    const int blocks = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    switch (dtype) {
#define SV_RA(D)                                                                              \
    case D:                                                                                   \
        hipLaunchKernelGGL(k_resize_adj<D>, dim3(blocks), dim3(256), 0, st, in, ipitch, icoff, \
                           Hf, Wf, Hc, Wc, C, mask, out, B);                                 \
        break;
        SV_RA(SV_F32)
        SV_RA(SV_BF16)
        SV_RA(SV_F16)
#undef SV_RA
    default: return SV_ERR_DTYPE;
    }
    SV_LAUNCH_CHECK("k_resize_adj");
    return SV_OK;
}

// ---------------------------------------------------------------------------
// Final layer adjoint.  With dY = 256 * dout at full resolution, per coarse
// pixel i and tap t = (u, v):
//   dT_t(i) = sum over full-res q inside of A(q, i) * dY(q - (u-1, v-1))
// (zero where q - delta leaves the image), then
//   dpre0[c](i) = lrelu'(G0[c](i)) * sum_t W_F[c][t] dT_t(i)   for c < c1.
// dT is written with 16 channels (9 used, the rest 0) for the weight gradient.
// ---------------------------------------------------------------------------
template <int DT>
__global__ void k_final_bwd(const float *__restrict__ dout, int H, int W, int h, int w, int B,
                            const void *__restrict__ wF, int wf_pitch, int c1,
                            const void *__restrict__ G0, float *__restrict__ dT,
                            float *__restrict__ dpre0)
{
    const size_t n = (size_t)B * h * w;
    for (size_t pix = blockIdx.x * (size_t)blockDim.x + threadIdx.x; pix < n;
         pix += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(pix % w), i = (int)((pix / w) % h), b = (int)(pix / ((size_t)w * h));
        const int ylo = max(0, ((i - 1) * H) / h - 1), yhi = min(H - 1, ((i + 2) * H) / h + 1);
        const int xlo = max(0, ((j - 1) * W) / w - 1), xhi = min(W - 1, ((j + 2) * W) / w + 1);
        float t[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) t[k] = 0.f;
        const float *db = dout + (size_t)b * H * W;
        for (int Y = ylo; Y <= yhi; ++Y) {
            const float wy = bilin_weight_to(Y, h, H, i);
            if (wy == 0.f) continue;
            for (int X = xlo; X <= xhi; ++X) {
                const float wx = bilin_weight_to(X, w, W, j);
                if (wx == 0.f) continue;
                const float wgt = 256.0f * wy * wx;
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    const int py = Y - (u - 1);
                    if (py < 0 || py >= H) continue;
#pragma unroll
                    for (int v = 0; v < 3; ++v) {
                        const int px = X - (v - 1);
                        if (px < 0 || px >= W) continue;
                        t[u * 3 + v] += wgt * db[(size_t)py * W + px];
                    }
                }
            }
        }
        float *dt = dT + pix * 16;
#pragma unroll
        for (int k = 0; k < 16; ++k) dt[k] = k < 9 ? t[k] : 0.f;
        const float *wf = (const float *)wF;  // the final projection is always packed in FP32
        const typename Elem<DT>::T *g0 = (const typename Elem<DT>::T *)G0 + pix * c1;
        for (int c = 0; c < c1; ++c) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < 9; ++k) s += wf[(size_t)k * wf_pitch + c] * t[k];
            dpre0[pix * c1 + c] = s * (Elem<DT>::load(g0 + c) > 0.f ? 1.f : 0.1f);
        }
    }
}

// Reparameterisation and KL adjoint: from dz to d[mu | logvar].
__global__ void k_latent_bwd(const float *__restrict__ dz, const float *__restrict__ ml,
                             const float *__restrict__ eps, const float *__restrict__ extra,
                             int npix, int L, float klw, float *__restrict__ dml)
{
    const size_t n = (size_t)npix * L;
    const float inv = 1.0f / (float)n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t p = e / L;
        const int c = (int)(e - p * L);
        const float mu = ml[p * 2 * L + c], lv = ml[p * 2 * L + L + c];
        const float g = dz[e];
        float dlv = klw * 0.5f * (expf(lv) - 1.0f) * inv;
        if (eps) dlv += g * eps[e] * 0.5f * expf(0.5f * lv);
        float dmu = g + klw * mu * inv;
        if (extra) {
            dmu += extra[p * 2 * L + c];
            dlv += extra[p * 2 * L + L + c];
        }
        dml[p * 2 * L + c] = dmu;
        dml[p * 2 * L + L + c] = dlv;
    }
}

// Deterministic sum (fixed grid, fixed tree) of scale * x[0..n) into *out.
constexpr int SUM_BLOCKS = 256;
__global__ void __launch_bounds__(256) k_sum_partial(const float *__restrict__ x, int64_t n,
                                                     float *__restrict__ part)
{
    __shared__ float sh[256];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    float s = 0.f;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += x[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void __launch_bounds__(256) k_sum_final(const float *__restrict__ part, float scale,
                                                   float *__restrict__ out)
{
    __shared__ float sh[256];
    sh[threadIdx.x] = threadIdx.x < SUM_BLOCKS ? part[threadIdx.x] : 0.f;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = scale * sh[0];
}

// ---------------------------------------------------------------------------
// Workspace of the backward pass (after the forward part holding E1..E3, T).
// ---------------------------------------------------------------------------
struct BwdLayout {
    size_t dT, dpre0, dG1up, dpre1, dcat1, dpre2, dcat2, dpre3, dz, dML, dpreE3, dpreE2, dpreE1,
        sum, part, total;
};

static BwdLayout bwd_layout(const NetShape &ns, const Levels &lv, int B) {
    BwdLayout l;
    auto px = [&](int k) { return (size_t)B * lv.h[k] * lv.w[k]; };
    const int c1 = ns.c1, c2 = ns.c2, c3 = ns.c3, L = ns.L;
    size_t o = 0;
    auto take = [&](size_t floats) { size_t r = o; o = align256(o + floats * sizeof(float)); return r; };
    l.dT = take(px(0) * 16);
    l.dpre0 = take(px(0) * c1);
    l.dG1up = take(px(0) * c1);
    l.dpre1 = take(px(1) * c1);
    l.dcat1 = take(px(1) * (c2 + c1));
    l.dpre2 = take(px(2) * c2);
    l.dcat2 = take(px(2) * (c3 + c2));
    l.dpre3 = take(px(3) * c3);
    l.dz = take(px(3) * L);
    l.dML = take(px(3) * 2 * L);
    l.dpreE3 = take(px(3) * c3);
    l.dpreE2 = take(px(2) * c2);
    l.dpreE1 = take(px(1) * c1);
    l.sum = take(SUM_BLOCKS);
    // the partial sums of the largest weight gradient (layers run one after another)
    const int lvl_out[NLAYERS] = {1, 2, 3, 3, 3, 2, 1, 0, 0};
    size_t mx = 0;
    for (int li = 0; li < NLAYERS; ++li) {
        const LayerSpec &s = ns.ly[li];
        const int k = lvl_out[li];
        const int cout = li == L_F ? 9 : s.cout;
        const int ks = li == L_F ? 1 : s.k;
        const WgradPlan w = wgrad_plan(B, lv.h[k], lv.w[k], s.cin, cout, ks);
        const size_t f = wgrad_part_floats(w);
        if (f > mx) mx = f;
    }
    l.part = take(mx);
    l.total = o;
    return l;
}

size_t net_bwd_workspace(const NetShape &ns, const Levels &lv, int B) {
    return bwd_layout(ns, lv, B).total;
}

static ConvSrc bsrc(const void *p, int kind, int C, int pitch, int coff, int hs, int ws, int sdt) {
    ConvSrc s{};
    s.ptr = p; s.kind = kind; s.C = C; s.pitch = pitch; s.coff = coff; s.hs = hs; s.ws = ws;
    s.sdt = sdt;
    return s;
}

#define SV_TRY(x)                       \
    do {                                \
        sv_status r_ = (x);             \
        if (r_ != SV_OK) return r_;     \
    } while (0)

// Input gradient of layer li through the forward conv kernel and the adjoint pack.
static sv_status dgrad(const NetShape &ns, const void *packed, int li, ConvSrc dy, int B, int Hi,
                       int Wi, int cout_needed, float *out, int out_pitch, const float *add,
                       int add_pitch, int add_coff, const void *mask, int mask_pitch, hipStream_t st) {
    ConvParams p{};
    p.src[0] = dy;
    p.B = B; p.Hi = Hi; p.Wi = Wi; p.Ho = Hi; p.Wo = Wi;
    p.Cin = dy.C;
    p.Cout = cout_needed;
    p.cin_pad = ns.bcin_pad[li];
    p.n_pad = ns.bn_pad[li];
    p.wpk = (const char *)packed + ns.bw_off[li];
    p.out = out; p.out_pitch = out_pitch; p.out_f32 = 1;
    p.add = add; p.add_pitch = add_pitch; p.add_coff = add_coff;
    p.mask = mask; p.mask_pitch = mask_pitch;
    const int ks = ns.ly[li].k;
    const int cfg = cout_needed <= 16 ? 5 : (cout_needed <= 32 ? 2 : 0);
    return launch_conv(ns.dtype, ks, 1, cfg, p, st);
}

sv_status net_backward(const NetShape &ns, const void *packed, const void *saved, int B, int H,
                       int W, const float *eps, const float *dout, const float *dml_extra,
                       float klw, float *grad, void *ws, hipStream_t st) {
    const Levels lv = net_levels(ns, H, W);
    const ActLayout a = net_act_layout(ns, lv, B);
    const BwdLayout bl = bwd_layout(ns, lv, B);
    char *w = (char *)ws;
    char *bw = w + a.ws_fwd;
    const char *sv_ = (const char *)saved;
    auto F = [&](size_t off) { return (float *)(bw + off); };
    const int c1 = ns.c1, c2 = ns.c2, c3 = ns.c3, L = ns.L, dt = ns.dtype;
    const uint8_t *disp = (const uint8_t *)(sv_ + a.disp), *img = (const uint8_t *)(sv_ + a.img);
    const float *ML = (const float *)(sv_ + a.ML);
    const void *Z = sv_ + a.Z, *G3 = sv_ + a.G3, *G2 = sv_ + a.G2, *G1 = sv_ + a.G1, *G0 = sv_ + a.G0;
    void *E1 = w + a.E1, *E2 = w + a.E2, *E3 = w + a.E3;
    const int *h = lv.h, *wd = lv.w;
    const ConvSrc none{};
    ConvSrc x0{};
    x0.ptr = disp; x0.img = img; x0.kind = SRC_X0; x0.C = 2; x0.hs = h[0]; x0.ws = wd[0];
    x0.scale0 = (float)ns.f / 256.0f;
    auto T_ = [&](const void *p, int C, int k) { return bsrc(p, SRC_TENSOR, C, C, 0, h[k], wd[k], 0); };
    auto Rz = [&](const void *p, int C, int k) { return bsrc(p, SRC_RESIZE, C, C, 0, h[k], wd[k], 0); };
    auto Gf = [&](float *p, int C, int pitch, int k) { return bsrc(p, SRC_TENSOR, C, pitch, 0, h[k], wd[k], SDT_F32); };
    float *part = F(bl.part);
    float *gl[NLAYERS];
    for (int i = 0; i < NLAYERS; ++i) gl[i] = grad + ns.p_off[i];

    // ---- recompute the encoder ----------------------------------------------------
    {
        auto fwd = [&](int li, ConvSrc s, int ki, int ko, void *out, int cout) {
            ConvParams p{};
            p.src[0] = s;
            p.B = B; p.Hi = h[ki]; p.Wi = wd[ki]; p.Ho = h[ko]; p.Wo = wd[ko];
            p.Cin = s.C; p.Cout = cout;
            p.cin_pad = ns.cin_pad[li]; p.n_pad = ns.n_pad[li];
            p.wpk = (const char *)packed + ns.w_off[li];
            p.bias = (const float *)((const char *)packed + ns.b_off[li]);
            p.out = out; p.out_pitch = cout; p.act = 1;
            return launch_conv(dt, 3, 2, net_default_cfg(ns, li, B * h[ko] * wd[ko]), p, st);
        };
        SV_TRY(launch_enc1(dt, disp, img, (float)ns.f / 256.0f, B, h[0], wd[0], h[1], wd[1], c1,
                           (const char *)packed + ns.w_off[L_E1], ns.n_pad[L_E1], ns.cin_pad[L_E1],
                           (const float *)((const char *)packed + ns.b_off[L_E1]), E1, st));
        SV_TRY(fwd(L_E2, T_(E1, c1, 1), 1, 2, E2, c2));
        SV_TRY(fwd(L_E3, T_(E2, c2, 2), 2, 3, E3, c3));
    }

    // ---- final layer -----------------------------------------------------------------
    {
        const size_t n = (size_t)B * h[0] * wd[0];
        const int blocks = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
        const void *wF = (const char *)packed + ns.w_off[L_F];
        switch (dt) {
#define SV_FB(D)                                                                                    \
        case D:                                                                                     \
            hipLaunchKernelGGL(k_final_bwd<D>, dim3(blocks), dim3(256), 0, st, dout, H, W, h[0],    \
                               wd[0], B, wF, ns.cin_pad[L_F], c1, G0, F(bl.dT), F(bl.dpre0));      \
            break;
            SV_FB(SV_F32)
            SV_FB(SV_BF16)
            SV_FB(SV_F16)
#undef SV_FB
        default: return SV_ERR_DTYPE;
        }
        SV_LAUNCH_CHECK("k_final_bwd");
        // dW_F from X = [G0, x0] and dT (a 1x1 layer with the 9 taps as outputs), in FP32
        SV_TRY(wgrad_layer(SV_F32, 1, 1, bsrc(G0, SRC_TENSOR, c1, c1, 0, h[0], wd[0], 1 + dt), x0, B,
                           h[0], wd[0], h[0], wd[0], 9, F(bl.dT), 16, part, 1, gl[L_F], st));
        // db_F = 256 * sum(dout)
        hipLaunchKernelGGL(k_sum_partial, dim3(SUM_BLOCKS), dim3(256), 0, st, dout,
                           (int64_t)B * H * W, F(bl.sum));
        hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, F(bl.sum), 256.0f,
                           gl[L_F] + 9 * (c1 + 2));
        SV_LAUNCH_CHECK("k_sum");
    }

    // ---- G0: input [resize(G1), x0] at level 0 -------------------------------------
    SV_TRY(wgrad_layer(dt, 3, 1, Rz(G1, c1, 1), x0, B, h[0], wd[0], h[0], wd[0], c1, F(bl.dpre0), c1,
                       part, 0, gl[L_G0], st));
    SV_TRY(dgrad(ns, packed, L_G0, Gf(F(bl.dpre0), c1, c1, 0), B, h[0], wd[0], c1, F(bl.dG1up), c1,
                 nullptr, 0, 0, nullptr, 0, st));
    SV_TRY(launch_resize_adj(dt, F(bl.dG1up), c1, 0, h[0], wd[0], h[1], wd[1], c1, G1, F(bl.dpre1),
                             B, st));
    // ---- G1: input [resize(G2), E1] at level 1 ---------------------------------------
    SV_TRY(wgrad_layer(dt, 3, 1, Rz(G2, c2, 2), T_(E1, c1, 1), B, h[1], wd[1], h[1], wd[1], c1,
                       F(bl.dpre1), c1, part, 0, gl[L_G1], st));
    SV_TRY(dgrad(ns, packed, L_G1, Gf(F(bl.dpre1), c1, c1, 1), B, h[1], wd[1], c2 + c1, F(bl.dcat1),
                 c2 + c1, nullptr, 0, 0, nullptr, 0, st));
    SV_TRY(launch_resize_adj(dt, F(bl.dcat1), c2 + c1, 0, h[1], wd[1], h[2], wd[2], c2, G2,
                             F(bl.dpre2), B, st));
    // ---- G2: input [resize(G3), E2] at level 2 ---------------------------------------
    SV_TRY(wgrad_layer(dt, 3, 1, Rz(G3, c3, 3), T_(E2, c2, 2), B, h[2], wd[2], h[2], wd[2], c2,
                       F(bl.dpre2), c2, part, 0, gl[L_G2], st));
    SV_TRY(dgrad(ns, packed, L_G2, Gf(F(bl.dpre2), c2, c2, 2), B, h[2], wd[2], c3 + c2, F(bl.dcat2),
                 c3 + c2, nullptr, 0, 0, nullptr, 0, st));
    SV_TRY(launch_resize_adj(dt, F(bl.dcat2), c3 + c2, 0, h[2], wd[2], h[3], wd[3], c3, G3,
                             F(bl.dpre3), B, st));
    // ---- G3 = lrelu(conv1x1(z)) -------------------------------------------------------
    const ConvSrc zsrc = eps ? T_(Z, L, 3) : bsrc(ML, SRC_TENSOR, L, 2 * L, 0, h[3], wd[3], SDT_F32);
    SV_TRY(wgrad_layer(dt, 1, 1, zsrc, none, B, h[3], wd[3], h[3], wd[3], c3, F(bl.dpre3), c3, part,
                       0, gl[L_G3], st));
    SV_TRY(dgrad(ns, packed, L_G3, Gf(F(bl.dpre3), c3, c3, 3), B, h[3], wd[3], L, F(bl.dz), L,
                 nullptr, 0, 0, nullptr, 0, st));
    // ---- latent: reparameterisation and KL ----------------------------------------------
    {
        const int npix = B * h[3] * wd[3];
        const size_t n = (size_t)npix * L;
        const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
        hipLaunchKernelGGL(k_latent_bwd, dim3(blocks), dim3(256), 0, st, F(bl.dz), ML, eps,
                           dml_extra, npix, L, klw, F(bl.dML));
        SV_LAUNCH_CHECK("k_latent_bwd");
    }
    // ---- HEAD: [mu | logvar] = conv1x1(E3) -------------------------------------------
    SV_TRY(wgrad_layer(dt, 1, 1, T_(E3, c3, 3), none, B, h[3], wd[3], h[3], wd[3], 2 * L, F(bl.dML),
                       2 * L, part, 0, gl[L_HEAD], st));
    SV_TRY(dgrad(ns, packed, L_HEAD, Gf(F(bl.dML), 2 * L, 2 * L, 3), B, h[3], wd[3], c3,
                 F(bl.dpreE3), c3, nullptr, 0, 0, E3, c3, st));
    // ---- encoder (stride 2): input gradients through the zero-inserted view ------------
    SV_TRY(wgrad_layer(dt, 3, 2, T_(E2, c2, 2), none, B, h[2], wd[2], h[3], wd[3], c3, F(bl.dpreE3),
                       c3, part, 0, gl[L_E3], st));
    SV_TRY(dgrad(ns, packed, L_E3, bsrc(F(bl.dpreE3), SRC_ZINS, c3, c3, 0, h[3], wd[3], SDT_F32), B, h[2],
                 wd[2], c2, F(bl.dpreE2), c2, F(bl.dcat2), c3 + c2, c3, E2, c2, st));
    SV_TRY(wgrad_layer(dt, 3, 2, T_(E1, c1, 1), none, B, h[1], wd[1], h[2], wd[2], c2, F(bl.dpreE2),
                       c2, part, 0, gl[L_E2], st));
    SV_TRY(dgrad(ns, packed, L_E2, bsrc(F(bl.dpreE2), SRC_ZINS, c2, c2, 0, h[2], wd[2], SDT_F32), B, h[1],
                 wd[1], c1, F(bl.dpreE1), c1, F(bl.dcat1), c2 + c1, c2, E1, c1, st));
    SV_TRY(wgrad_layer(dt, 3, 2, x0, none, B, h[0], wd[0], h[1], wd[1], c1, F(bl.dpreE1), c1, part,
                       0, gl[L_E1], st));
    return SV_OK;
}

}  // namespace sv
