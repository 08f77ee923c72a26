// Network glue: the final upsampling layer and the reparameterisation.
#include <algorithm>
#include <mutex>

#include "kernels.h"

namespace sv {

// Final layer (Table I, "UP-SAMPLING"): R = conv3x3(resize([G0, x0] -> H x W))
// to one channel, plus the bilinear upscaling of the coarse map (the paper's
// "Mini+Linear" baseline, Sec. IV-C) as the residual base.  Convolution and
// resize are both linear, so with the per-tap projections
//   T_t(i) = sum_c W_F[c, t] X[c](i),  X = [G0, x0],  t = (u, v) in 3 x 3,
// computed at the coarse level,
//   R(Y, X) = sum_t [inside] resize(T_t)(Y + u - 1, X + v - 1).
// Bilinear resizing is separable as well, so the sum is taken in two passes:
//   S_v(Y, x) = sum_u [row Y + u - 1 inside] lerp_rows(T_uv)(Y + u - 1, x)
// on the coarse columns x, then
//   R(Y, X) = sum_v [column X + v - 1 inside] lerp_cols(S_v(Y, .))(X + v - 1).
//
// One workgroup = FIN_TILE_W x FIN_TILE_H output pixels and everything in
// LDS: the bilinear indices and weights of the tile's FIN_TILE_W + 2 columns
// and FIN_TILE_H + 2 rows (the 3 x 3 neighbourhood reaches one pixel past
// each edge), the 9 projections T and the coarse disparity on the coarse
// window the tile touches (T computed there from G0 and x0 with the FP32
// weights), then S.  For o in a run of K + 1 consecutive output positions
// (K = tile + 1) the lower bilinear index grows by at most ceil(K n_in / n_out),
// so with n_in = ceil(n_out / f) the window spans at most ceil(K / f) + 3 coarse
// positions, and never more than K + 2: fin_window() gives that bound and
// sizes the dynamic LDS.
constexpr int FIN_CX = FIN_TILE_W + 2, FIN_CY = FIN_TILE_H + 2;
constexpr int FIN_THREADS = 256;
static_assert(FIN_TILE_W == 64 && FIN_TILE_H % (FIN_THREADS / 64) == 0, "final tile shape");

static inline void fin_window(int f, int &ph, int &pw) {
    ph = std::min(FIN_TILE_H + 3, cdiv(FIN_TILE_H + 1, f) + 3);
    pw = std::min(FIN_TILE_W + 3, cdiv(FIN_TILE_W + 1, f) + 3);
}
// dynamic LDS (floats): T[9][ph][pw], d[ph][pw], S[FIN_TILE_H][3][pw], D[FIN_TILE_H][pw]
static inline size_t fin_lds_bytes(int f) {
    int ph, pw;
    fin_window(f, ph, pw);
    return sizeof(float) * ((size_t)10 * ph * pw + (size_t)4 * FIN_TILE_H * pw);
}

struct FinTab {
    int cx0[FIN_CX], cx1[FIN_CX], cy0[FIN_CY], cy1[FIN_CY];  // -1: outside the image (final_tile)
    float clx[FIN_CX], cly[FIN_CY];
    float cwx[FIN_CX], cwy[FIN_CY];  // gather_tile: weight of the lower corner, 0 outside the image
};

// Loads 8 consecutive stored channels as FP32.
template <int DT>
__device__ __forceinline__ void load8(const typename Elem<DT>::T *p, float (&v)[8]) {
    if constexpr (DT == SV_F32) {
        const f32x4 a = *(const f32x4 *)p, b = *(const f32x4 *)(p + 4);
        v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3];
        v[4] = b[0]; v[5] = b[1]; v[6] = b[2]; v[7] = b[3];
    } else {
        const u16x8 q = *(const u16x8 *)p;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = Elem<DT>::load((const typename Elem<DT>::T *)&q + i);
    }
}

// q / d for 0 <= q < 8192 and 1 <= d <= 160 from inv = 1.0f / d (correctly
// rounded): (q + 1/2) / d stays at least 1 / (2d) away from an integer, far
// more than the rounding of the product (checked exhaustively for that range).
__device__ __forceinline__ int fin_div(int q, float inv) { return (int)(((float)q + 0.5f) * inv); }

// PRE: the nine projections are read from Tpre (FP32 [9][plane] at the
// image's pixel offset; G0, ib and wF unused) instead of computed here.
template <int DT, bool PRE = false>
__device__ __forceinline__ void final_tile(float *dyn, FinTab &tb, int PHm, int PWm,
                                           const typename Elem<DT>::T *__restrict__ G0, int c1,
                                           const uint8_t *__restrict__ db,
                                           const uint8_t *__restrict__ ib,
                                           const float *__restrict__ wF, int wf_pitch,
                                           float scale0, float bias, int h, int w, int H, int W,
                                           int X0, int Y0, float *__restrict__ out,
                                           const float *__restrict__ Tpre = nullptr, long long plane = 0)
{
    const int tid = threadIdx.x;
    float *sT = dyn;                           // [9][PHm][PWm]
    float *sd = sT + 9 * PHm * PWm;            // [PHm][PWm]
    float *sS = sd + PHm * PWm;                // [FIN_TILE_H][3][PWm]
    float *sD = sS + FIN_TILE_H * 3 * PWm;     // [FIN_TILE_H][PWm]
    // coarse window: from the lower index of the first column / row in range to
    // the upper index of the last
    int xa, ya, xb, yb, i1;
    float lam;
    bilin(max(X0 - 1, 0), w, W, xa, i1, lam);
    bilin(max(Y0 - 1, 0), h, H, ya, i1, lam);
    bilin(min(X0 + FIN_TILE_W, W - 1), w, W, i1, xb, lam);
    bilin(min(Y0 + FIN_TILE_H, H - 1), h, H, i1, yb, lam);
    const int pw = xb - xa + 1, ph = yb - ya + 1;
    if (ph > PHm || pw > PWm) return;  // excluded by the window bound
    if (tid < FIN_CX) {
        const int X = X0 - 1 + tid;
        int x0 = -1, x1 = -1;
        float lx = 0.f;
        if (X >= 0 && X < W) {
            bilin(X, w, W, x0, x1, lx);
            x0 -= xa;
            x1 -= xa;
        }
        tb.cx0[tid] = x0;
        tb.cx1[tid] = x1;
        tb.clx[tid] = lx;
    } else if (tid >= 128 && tid < 128 + FIN_CY) {
        const int r = tid - 128, Y = Y0 - 1 + r;
        int y0 = -1, y1 = -1;
        float ly = 0.f;
        if (Y >= 0 && Y < H) {
            bilin(Y, h, H, y0, y1, ly);
            y0 -= ya;
            y1 -= ya;
        }
        tb.cy0[r] = y0;
        tb.cy1[r] = y1;
        tb.cly[r] = ly;
    }
    // T and the coarse disparity on the window.  Work item = one coarse pixel:
    // its channels are loaded once, 32 at a time (all in flight before any
    // product), and feed the nine tap projections as fused multiply-adds; the
    // weights are the same for every thread (scalar loads).
    const float inv_pw = 1.0f / (float)pw;
    const int npx = ph * pw;
    if constexpr (PRE) {
        // nine planes and the coarse disparity on the window, loads first
        for (int q = tid; q < npx; q += FIN_THREADS) {
            const int r = fin_div(q, inv_pw), c = q - r * pw;
            const size_t gp = (size_t)(ya + r) * w + xa + c;
            float a[9];
#pragma unroll
            for (int t = 0; t < 9; ++t) a[t] = Tpre[t * plane + gp];
            const float dv = (float)db[gp];
#pragma unroll
            for (int t = 0; t < 9; ++t) sT[(t * PHm + r) * PWm + c] = a[t];
            sd[r * PWm + c] = dv;
        }
    }
    for (int q = PRE ? npx : tid; q < npx; q += FIN_THREADS) {
        const int r = fin_div(q, inv_pw), c = q - r * pw;
        const size_t gp = (size_t)(ya + r) * w + xa + c;
        const float dv = (float)db[gp];
        const float x0d = scale0 * dv, x0i = (float)ib[gp] * (1.0f / 256.0f);
        const typename Elem<DT>::T *g = G0 + gp * c1;
        float a[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) a[t] = 0.f;
        for (int c0 = 0; c0 < c1; c0 += 32) {
            float v[32];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (c0 + 8 * k < c1) {
                    float u[8];
                    load8<DT>(g + c0 + 8 * k, u);
#pragma unroll
                    for (int i = 0; i < 8; ++i) v[8 * k + i] = u[i];
                } else {
#pragma unroll
                    for (int i = 0; i < 8; ++i) v[8 * k + i] = 0.f;
                }
            }
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const float *wt = wF + (size_t)t * wf_pitch + c0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (c0 + 8 * k < c1) {
#pragma unroll
                        for (int i = 0; i < 8; ++i) a[t] = fmaf(wt[8 * k + i], v[8 * k + i], a[t]);
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const float *wt = wF + (size_t)t * wf_pitch + c1;
            a[t] = fmaf(wt[1], x0i, fmaf(wt[0], x0d, a[t]));
            sT[(t * PHm + r) * PWm + c] = a[t];
        }
        sd[r * PWm + c] = dv;
    }
    __syncthreads();
    // vertical pass: S_v(Y, x) and the residual base's row interpolation D(Y, x)
    for (int e = tid; e < FIN_TILE_H * 4 * pw; e += FIN_THREADS) {
        const int rr = fin_div(e, inv_pw), c = e - rr * pw;
        const int ty = rr >> 2, v = rr & 3;
        if (v < 3) {
            float s = 0.f;
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int y0 = tb.cy0[ty + u];
                if (y0 < 0) continue;
                const int y1 = tb.cy1[ty + u];
                const float ly = tb.cly[ty + u];
                const float *tt = sT + (u * 3 + v) * PHm * PWm;
                s += (1.f - ly) * tt[y0 * PWm + c] + ly * tt[y1 * PWm + c];
            }
            sS[(ty * 3 + v) * PWm + c] = s;
        } else {
            const int y0 = tb.cy0[ty + 1];
            float s = 0.f;
            if (y0 >= 0) {
                const int y1 = tb.cy1[ty + 1];
                const float ly = tb.cly[ty + 1];
                s = (1.f - ly) * sd[y0 * PWm + c] + ly * sd[y1 * PWm + c];
            }
            sD[ty * PWm + c] = s;
        }
    }
    __syncthreads();
    // horizontal pass, one output pixel per thread and row; a thread keeps one
    // column, so its three column taps are read from the table once
    const int tx = tid & 63;
    const int X = X0 + tx;
    int hx0[3], hx1[3];
    float hlx[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        hx0[v] = tb.cx0[tx + v];
        hx1[v] = tb.cx1[tx + v];
        hlx[v] = tb.clx[tx + v];
    }
#pragma unroll
    for (int ty = tid >> 6; ty < FIN_TILE_H; ty += FIN_THREADS / 64) {
        const int Y = Y0 + ty;
        if (X < W && Y < H) {
            float acc = bias;
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                if (hx0[v] < 0) continue;
                const float *ss = sS + (ty * 3 + v) * PWm;
                acc += (1.f - hlx[v]) * ss[hx0[v]] + hlx[v] * ss[hx1[v]];
            }
            const float *dd = sD + ty * PWm;
            const float base = scale0 * ((1.f - hlx[1]) * dd[hx0[1]] + hlx[1] * dd[hx1[1]]);
            out[(size_t)Y * W + X] = 256.0f * (acc + base);
        }
    }
    __syncthreads();  // the LDS is reused by the next tile of a persistent loop
}

template <int DT>
__global__ void __launch_bounds__(FIN_THREADS)
k_final(const typename Elem<DT>::T *__restrict__ G0, int c1, const uint8_t *__restrict__ disp,
        const uint8_t *__restrict__ img, const float *__restrict__ wF, int wf_pitch, float scale0,
        const float *__restrict__ biasF, int h, int w, int H, int W, int PHm, int PWm,
        float *__restrict__ out)
{
    extern __shared__ __attribute__((aligned(16))) float fin_dyn[];
    __shared__ FinTab tb;
    const int b = blockIdx.z;
    const size_t o = (size_t)b * h * w;
    final_tile<DT>(fin_dyn, tb, PHm, PWm, G0 + o * c1, c1, disp + o, img + o, wF, wf_pitch, scale0,
                   biasF[0], h, w, H, W, blockIdx.x * FIN_TILE_W, blockIdx.y * FIN_TILE_H,
                   out + (size_t)b * H * W);
}

// Persistent variant over the pair table; each pair writes its own output map.
template <int DT>
__global__ void __launch_bounds__(FIN_THREADS)
k_final_tab(const PairTable *__restrict__ tab, const typename Elem<DT>::T *__restrict__ G0, int c1,
            const uint8_t *__restrict__ disp, const uint8_t *__restrict__ img,
            const float *__restrict__ wF, int wf_pitch, float scale0,
            const float *__restrict__ biasF, int PHm, int PWm)
{
    extern __shared__ __attribute__((aligned(16))) float fin_dyn[];
    __shared__ FinTab tb;
    const int n = tab->n;
    const int *cum = tab->cum[BS_FINAL];
    const int total = cum[n];
    const float bias = biasF[0];
    // round k takes tiles k G .. k G + G - 1 (G = gridDim.x); hardware id i
    // takes tile (i % 8) (G / 8) + i / 8 of the round, so that each XCD covers
    // a contiguous run of tiles (workgroups go round robin to the XCDs)
    const int G = (int)gridDim.x, q8 = G / 8, hw = (int)blockIdx.x;
    const int lid = hw < 8 * q8 ? (hw % 8) * q8 + hw / 8 : hw;
    for (int t = lid; t < total; t += G) {
        const int i = table_find(cum, n, t);
        const PairGeo &g = tab->pair[i];
        const int local = t - cum[i];
        const int tx = cdiv_d(g.W, FIN_TILE_W);
        const size_t o = (size_t)g.off[0];
        final_tile<DT>(fin_dyn, tb, PHm, PWm, G0 + o * c1, c1, disp + o, img + o, wF, wf_pitch,
                       scale0, bias, g.h[0], g.w[0], g.H, g.W, (local % tx) * FIN_TILE_W,
                       (local / tx) * FIN_TILE_H, g.out);
    }
}

// The gather from precomputed projections T (FP32 [9][plane]).  Tiles are
// FIN_TILE_W x TH output pixels, TH = gather_tile_h(f, output pixels): taller
// tiles at larger f, where a coarse window row covers more output rows, so
// that the window's halo is re-read less, while there are enough of them to
// fill the GPU.  Horizontal pass, per coarse row i of the
// window and row tap u, by a thread that owns output column X (it keeps the
// column indices and weights of X - 1, X, X + 1, zero outside the image: the
// 3 x 3 convolution's padding of the resized map):
//   H_u(i, X) = sum_v [(1 - lx_v) T_uv(i, x0_v) + lx_v T_uv(i, x1_v)],
// and the base's H_d(i, X) from the coarse disparity at column X; vertical
// pass, four adjacent output pixels per thread (one 16-byte store):
//   R(Y, X) = sum_u [(1 - ly_u) H_u(y0_u, X) + ly_u H_u(y1_u, X)],
//   out = 256 (bias + R + f d(Y, X) / 256).
// Dynamic LDS (floats): T[9][PHm][PWm], d[PHm][PWm], H[4][PHm][FIN_TILE_W].
int gather_tile_h(int f, long long out_px) {
    int th = f >= 4 ? 64 : (f >= 2 ? 32 : 16);
    while (th > 16 && out_px < 1024LL * FIN_TILE_W * th) th /= 2;
    return th;
}

static inline void gather_window(int f, int th, int &ph, int &pw) {
    ph = std::min(th + 3, cdiv(th + 1, f) + 3);
    pw = std::min(FIN_TILE_W + 3, cdiv(FIN_TILE_W + 1, f) + 3);
}

static inline size_t gather_lds_bytes(int f, int th) {
    int ph, pw;
    gather_window(f, th, ph, pw);
    return sizeof(float) * ((((size_t)10 * ph * pw + 3) & ~(size_t)3) + (size_t)4 * ph * FIN_TILE_W);
}

template <int TH>
struct GatherTab {
    int cx0[FIN_CX], cx1[FIN_CX], cy0[TH + 2], cy1[TH + 2];
    float clx[FIN_CX], cwx[FIN_CX], cly[TH + 2], cwy[TH + 2];  // cw: weight of the lower corner, 0 outside
};

typedef float f32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

// The coarse window [ya, ya + ph) x [xa, xa + pw) that the tile at (X0, Y0)
// reads (its 3 x 3 neighbourhood reaches one output pixel past each edge).
struct GatherWin {
    int xa, ya, pw, ph;
};

template <int TH>
__device__ __forceinline__ GatherWin gather_win(int h, int w, int H, int W, int X0, int Y0) {
    GatherWin g;
    int xb, yb, i1;
    float lam;
    bilin(max(X0 - 1, 0), w, W, g.xa, i1, lam);
    bilin(max(Y0 - 1, 0), h, H, g.ya, i1, lam);
    bilin(min(X0 + FIN_TILE_W, W - 1), w, W, i1, xb, lam);
    bilin(min(Y0 + TH, H - 1), h, H, i1, yb, lam);
    g.pw = xb - g.xa + 1;
    g.ph = yb - g.ya + 1;
    return g;
}

// The tile's column and row tables: source indices relative to the window,
// bilinear weights, and zero weights outside the image.
template <int TH>
__device__ __forceinline__ void gather_tables(GatherTab<TH> &tb, const GatherWin &g, int h, int w, int H,
                                              int W, int X0, int Y0) {
    const int tid = threadIdx.x;
    if (tid < FIN_CX) {
        const int X = X0 - 1 + tid;
        int x0 = 0, x1 = 0;
        float lx = 0.f, wx = 0.f;
        if (X >= 0 && X < W) {
            bilin(X, w, W, x0, x1, lx);
            x0 -= g.xa;
            x1 -= g.xa;
            wx = 1.f - lx;
        }
        tb.cx0[tid] = x0;
        tb.cx1[tid] = x1;
        tb.clx[tid] = lx;
        tb.cwx[tid] = wx;
    } else if (tid >= 128 && tid < 128 + TH + 2) {
        const int r = tid - 128, Y = Y0 - 1 + r;
        int y0 = 0, y1 = 0;
        float ly = 0.f, wy = 0.f;
        if (Y >= 0 && Y < H) {
            bilin(Y, h, H, y0, y1, ly);
            y0 -= g.ya;
            y1 -= g.ya;
            wy = 1.f - ly;
        }
        tb.cy0[r] = y0;
        tb.cy1[r] = y1;
        tb.cly[r] = ly;
        tb.cwy[r] = wy;
    }
}

// One round of the window's loads: window pixels q0 and q0 + FIN_THREADS, the
// nine projections and the coarse disparity of each (past the window's end
// the last pixel is read again and not stored).
struct GatherRound {
    float a[2][10];
    int rr[2], cc[2];
};

__device__ __forceinline__ void gather_fetch(GatherRound &R, const float *__restrict__ Tp, long long plane,
                                             const uint8_t *__restrict__ db, int w, const GatherWin &g,
                                             int q0) {
    const float inv_pw = 1.0f / (float)g.pw;
    const int npx = g.ph * g.pw;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int q = min(q0 + k * FIN_THREADS, npx - 1);
        R.rr[k] = fin_div(q, inv_pw);
        R.cc[k] = q - R.rr[k] * g.pw;
        const size_t gp = (size_t)(g.ya + R.rr[k]) * w + g.xa + R.cc[k];
#pragma unroll
        for (int t = 0; t < 9; ++t) R.a[k][t] = Tp[t * plane + gp];
        R.a[k][9] = (float)db[gp];
    }
}

__device__ __forceinline__ void gather_put(const GatherRound &R, float *sT, float *sd, int PHm, int PWm,
                                           int npx, int q0) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (q0 + k * FIN_THREADS < npx) {
#pragma unroll
            for (int t = 0; t < 9; ++t) sT[(t * PHm + R.rr[k]) * PWm + R.cc[k]] = R.a[k][t];
            sd[R.rr[k] * PWm + R.cc[k]] = R.a[k][9];
        }
    }
}

// The two passes over a staged window (the LDS holds T, d and the tables),
// then the stores; ends with a barrier, so the LDS can take the next tile.
template <int TH>
__device__ __forceinline__ void gather_passes(float *dyn, const GatherTab<TH> &tb, int PHm, int PWm, int ph,
                                              float scale0, float bias, int H, int W, int X0, int Y0,
                                              float *__restrict__ out)
{
    const int tid = threadIdx.x;
    const float *sT = dyn;                   // [9][PHm][PWm]
    const float *sd = sT + 9 * PHm * PWm;    // [PHm][PWm]
    float *sH = dyn + ((10 * PHm * PWm + 3) & ~3);  // [4][PHm][FIN_TILE_W], 16-byte aligned
    {
        const int tx = tid & (FIN_TILE_W - 1), rg = tid / FIN_TILE_W;
        constexpr int NRG = FIN_THREADS / FIN_TILE_W;
        // this column's taps: X - 1, X, X + 1 are table entries tx, tx + 1, tx + 2
        int hx0[3], hx1[3];
        float hl[3], hw[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            hx0[v] = tb.cx0[tx + v];
            hx1[v] = tb.cx1[tx + v];
            hl[v] = tb.clx[tx + v];
            hw[v] = tb.cwx[tx + v];
        }
        for (int i = rg; i < ph; i += NRG) {
            float hu[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                float acc = 0.f;
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    const float *row = sT + ((u * 3 + v) * PHm + i) * PWm;
                    acc = fmaf(hw[v], row[hx0[v]], acc);
                    acc = fmaf(hl[v], row[hx1[v]], acc);
                }
                hu[u] = acc;
            }
            const float *drow = sd + i * PWm;
            const float hd = fmaf(hl[1], drow[hx1[1]], hw[1] * drow[hx0[1]]);
#pragma unroll
            for (int u = 0; u < 3; ++u) sH[(u * PHm + i) * FIN_TILE_W + tx] = hu[u];
            sH[(3 * PHm + i) * FIN_TILE_W + tx] = hd;
        }
    }
    __syncthreads();
    constexpr int QW = FIN_TILE_W / 4;  // threads per output row
    const int c4 = (tid % QW) * 4, X = X0 + c4;
    for (int ty = tid / QW; ty < TH; ty += FIN_THREADS / QW) {
        const int Y = Y0 + ty;
        if (Y >= H || X >= W) continue;
        f32x4 acc = {bias, bias, bias, bias};
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int e = ty + u;  // table entry of row Y + u - 1
            const float *hp = sH + u * PHm * FIN_TILE_W + c4;
            const f32x4 h0 = *(const f32x4 *)(hp + tb.cy0[e] * FIN_TILE_W);
            const f32x4 h1 = *(const f32x4 *)(hp + tb.cy1[e] * FIN_TILE_W);
            const float wy = tb.cwy[e], ly = tb.cly[e];
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] = fmaf(ly, h1[k], fmaf(wy, h0[k], acc[k]));
        }
        const int e = ty + 1;
        const float *dp = sH + 3 * PHm * FIN_TILE_W + c4;
        const f32x4 d0 = *(const f32x4 *)(dp + tb.cy0[e] * FIN_TILE_W);
        const f32x4 d1 = *(const f32x4 *)(dp + tb.cy1[e] * FIN_TILE_W);
        f32x4 r;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float base = fmaf(tb.cly[e], d1[k], tb.cwy[e] * d0[k]);
            r[k] = 256.0f * fmaf(scale0, base, acc[k]);
        }
        float *op = out + (size_t)Y * W + X;
        if (X + 3 < W) {
            // rows of odd W are not 16-byte aligned: relies on unaligned global access
            *(f32x4_a4 *)op = f32x4_a4{r[0], r[1], r[2], r[3]};
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (X + k < W) op[k] = r[k];
        }
    }
    __syncthreads();  // the LDS is reused by the next tile of a persistent loop
}

template <int TH>
__device__ __forceinline__ void gather_tile(float *dyn, GatherTab<TH> &tb, int PHm, int PWm,
                                            const float *__restrict__ Tp, long long plane,
                                            const uint8_t *__restrict__ db, float scale0, float bias,
                                            int h, int w, int H, int W, int X0, int Y0,
                                            float *__restrict__ out)
{
    const GatherWin g = gather_win<TH>(h, w, H, W, X0, Y0);
    if (g.ph > PHm || g.pw > PWm) return;  // excluded by the window bound
    gather_tables<TH>(tb, g, h, w, H, W, X0, Y0);
    // the nine projections and the coarse disparity on the window; two
    // window pixels per thread and round, all of their loads issued first
    float *sT = dyn, *sd = dyn + 9 * PHm * PWm;
    const int npx = g.ph * g.pw;
    for (int q0 = threadIdx.x; q0 < npx; q0 += 2 * FIN_THREADS) {
        GatherRound R;
        gather_fetch(R, Tp, plane, db, w, g, q0);
        gather_put(R, sT, sd, PHm, PWm, npx, q0);
    }
    __syncthreads();
    gather_passes<TH>(dyn, tb, PHm, PWm, g.ph, scale0, bias, H, W, X0, Y0, out);
}

// The gather from precomputed projections (uniform batch and pair table).
template <int TH>
__global__ void __launch_bounds__(FIN_THREADS)
k_final_gather(const float *__restrict__ T, long long plane, const uint8_t *__restrict__ disp, float scale0,
               const float *__restrict__ biasF, int h, int w, int H, int W, int PHm, int PWm,
               float *__restrict__ out)
{
    extern __shared__ __attribute__((aligned(16))) float fin_dyn[];
    __shared__ GatherTab<TH> tb;
    // XCD-aware order (workgroups go round robin to the eight XCDs, each with
    // its own L2): hardware id i takes tile (i % 8) q + i / 8, q = N / 8, so
    // each XCD covers a contiguous run of tiles and the windows' overlapping
    // rows and columns are re-read from its own L2
    const int gx = (int)gridDim.x, gy = (int)gridDim.y;
    const int nblk = gx * gy * (int)gridDim.z;
    const int hw = (int)blockIdx.x + gx * ((int)blockIdx.y + gy * (int)blockIdx.z);
    const int q8 = nblk / 8;
    const int lid = hw < 8 * q8 ? (hw % 8) * q8 + hw / 8 : hw;
    const int b = lid / (gx * gy), rem = lid - b * (gx * gy);
    const int by = rem / gx, bx = rem - by * gx;
    const size_t o = (size_t)b * h * w;
    gather_tile<TH>(fin_dyn, tb, PHm, PWm, T + o, plane, disp + o, scale0, biasF[0], h, w, H, W,
                    bx * FIN_TILE_W, by * TH, out + (size_t)b * H * W);
}

template <int TH>
__global__ void __launch_bounds__(FIN_THREADS)
k_final_gather_tab(const PairTable *__restrict__ tab, const float *__restrict__ T, long long plane,
                   const uint8_t *__restrict__ disp, float scale0, const float *__restrict__ biasF, int PHm,
                   int PWm)
{
    extern __shared__ __attribute__((aligned(16))) float fin_dyn[];
    __shared__ GatherTab<TH> tb;
    const int n = tab->n;
    const int *cum = tab->cum[BS_FINAL];
    const int total = cum[n];
    const float bias = biasF[0];
    // round k takes tiles k G .. k G + G - 1 (G = gridDim.x); hardware id i
    // takes tile (i % 8) (G / 8) + i / 8 of the round, so that each XCD covers
    // a contiguous run of tiles (workgroups go round robin to the XCDs)
    const int G = (int)gridDim.x, q8 = G / 8, hw = (int)blockIdx.x;
    const int lid = hw < 8 * q8 ? (hw % 8) * q8 + hw / 8 : hw;
    for (int t = lid; t < total; t += G) {
        const int i = table_find(cum, n, t);
        const PairGeo &g = tab->pair[i];
        const int local = t - cum[i];
        const int tx = cdiv_d(g.W, FIN_TILE_W);
        const size_t o = (size_t)g.off[0];
        gather_tile<TH>(fin_dyn, tb, PHm, PWm, T + o, plane, disp + o, scale0, bias, g.h[0], g.w[0], g.H, g.W,
                        (local % tx) * FIN_TILE_W, (local / tx) * TH, g.out);
    }
}

// The dynamic LDS of the final layer stays under 80 KB (f = 1); the kernels
// are allowed that much once, before their first launch.
static sv_status fin_allow_lds() {
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        const int bytes = 96 * 1024;
        const void *fns[12] = {(const void *)k_final<SV_F32>,          (const void *)k_final<SV_BF16>,
                               (const void *)k_final<SV_F16>,          (const void *)k_final_tab<SV_F32>,
                               (const void *)k_final_tab<SV_BF16>,     (const void *)k_final_tab<SV_F16>,
                               (const void *)k_final_gather<16>,       (const void *)k_final_gather_tab<16>,
                               (const void *)k_final_gather<32>,       (const void *)k_final_gather_tab<32>,
                               (const void *)k_final_gather<64>,       (const void *)k_final_gather_tab<64>};
        for (const void *fn : fns) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            if (e != hipSuccess && err == hipSuccess) err = e;
        }
    });
    if (err != hipSuccess) return hip_fail(err, "hipFuncSetAttribute(k_final)");
    return SV_OK;
}

sv_status launch_final_tab(const PairTable *tab, int grid, int dtype, const void *G0, int c1,
                           const uint8_t *disp, const uint8_t *img, const float *wF, int wf_pitch,
                           int f, const float *biasF, hipStream_t s)
{
    if (sv_status r = fin_allow_lds(); r != SV_OK) return r;
    int PHm, PWm;
    fin_window(f, PHm, PWm);
    const size_t lds = fin_lds_bytes(f);
    const float scale0 = (float)f / 256.0f;
    switch (dtype) {
#define SV_FT(D)                                                                                      \
    case D:                                                                                           \
        hipLaunchKernelGGL(k_final_tab<D>, dim3((unsigned)resident_grid((const void *)k_final_tab<D>, lds, grid)), \
                           dim3(FIN_THREADS), lds, s, tab,                                            \
                           (const typename Elem<D>::T *)G0, c1, disp, img, wF, wf_pitch, scale0,      \
                           biasF, PHm, PWm);                                                          \
        break;
        SV_FT(SV_F32)
        SV_FT(SV_BF16)
        SV_FT(SV_F16)
#undef SV_FT
    default: return SV_ERR_DTYPE;
    }
    SV_LAUNCH_CHECK("k_final_tab");
    return SV_OK;
}

sv_status launch_final(int dtype, const void *G0, int c1, const uint8_t *disp, const uint8_t *img,
                       const float *wF, int wf_pitch, int f, const float *biasF, int B, int h,
                       int w, int H, int W, float *out, hipStream_t s)
{
    if (sv_status r = fin_allow_lds(); r != SV_OK) return r;
    int PHm, PWm;
    fin_window(f, PHm, PWm);
    const size_t lds = fin_lds_bytes(f);
    const float scale0 = (float)f / 256.0f;
    dim3 grid(cdiv(W, FIN_TILE_W), cdiv(H, FIN_TILE_H), B);
    switch (dtype) {
#define SV_FU(D)                                                                                      \
    case D:                                                                                           \
        hipLaunchKernelGGL(k_final<D>, grid, dim3(FIN_THREADS), lds, s,                               \
                           (const typename Elem<D>::T *)G0, c1, disp, img, wF, wf_pitch, scale0,      \
                           biasF, h, w, H, W, PHm, PWm, out);                                         \
        break;
        SV_FU(SV_F32)
        SV_FU(SV_BF16)
        SV_FU(SV_F16)
#undef SV_FU
    default: return SV_ERR_DTYPE;
    }
    SV_LAUNCH_CHECK("k_final");
    return SV_OK;
}

sv_status launch_final_gather(const float *T, long long plane, const uint8_t *disp, int f,
                              const float *biasF, int B, int h, int w, int H, int W, float *out,
                              hipStream_t s)
{
    if (sv_status r = fin_allow_lds(); r != SV_OK) return r;
    const int th = gather_tile_h(f, (long long)B * H * W);
    int PHm, PWm;
    gather_window(f, th, PHm, PWm);
    dim3 grid(cdiv(W, FIN_TILE_W), cdiv(H, th), B);
#define SV_FG(TH)                                                                                         \
    hipLaunchKernelGGL(k_final_gather<TH>, grid, dim3(FIN_THREADS), gather_lds_bytes(f, th), s, T, plane, disp, \
                       (float)f / 256.0f, biasF, h, w, H, W, PHm, PWm, out)
    if (th == 64) SV_FG(64);
    else if (th == 32) SV_FG(32);
    else SV_FG(16);
#undef SV_FG
    SV_LAUNCH_CHECK("k_final_gather");
    return SV_OK;
}

sv_status launch_final_gather_tab(const PairTable *tab, int grid, const float *T, long long plane,
                                  const uint8_t *disp, int f, int th, const float *biasF, hipStream_t s)
{
    if (sv_status r = fin_allow_lds(); r != SV_OK) return r;
    if (th != 16 && th != 32 && th != 64) return SV_ERR_RANGE;
    int PHm, PWm;
    gather_window(f, th, PHm, PWm);
#define SV_FG(TH)                                                                                          \
    hipLaunchKernelGGL(k_final_gather_tab<TH>,                                                             \
                       dim3((unsigned)resident_grid((const void *)k_final_gather_tab<TH>, gather_lds_bytes(f, th), grid)), \
                       dim3(FIN_THREADS), gather_lds_bytes(f, th), s, tab, T, plane, disp, (float)f / 256.0f, biasF, PHm, PWm)
    if (th == 64) SV_FG(64);
    else if (th == 32) SV_FG(32);
    else SV_FG(16);
#undef SV_FG
    SV_LAUNCH_CHECK("k_final_gather_tab");
    return SV_OK;
}

// Reparameterisation, Eq. (8) in the standard form: z = mu + eps * exp(logvar / 2),
// from the FP32 head output [.. ][mu | logvar] into the compute dtype.
template <int DT>
__global__ void k_reparam(const float *__restrict__ ml, const float *__restrict__ eps, int npix,
                          int L, typename Elem<DT>::T *__restrict__ z)
{
    const size_t n = (size_t)npix * L;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t p = e / L;
        const int c = (int)(e - p * L);
        const float mu = ml[p * 2 * L + c], lv = ml[p * 2 * L + L + c];
        z[e] = Elem<DT>::make(mu + eps[e] * expf(0.5f * lv));
    }
}

sv_status launch_reparam(const float *ml, const float *eps, int npix, int L, void *z, int dtype,
                         hipStream_t s)
{
    const size_t n = (size_t)npix * L;
    const int blocks = (int)((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048);
    switch (dtype) {
    case SV_F32:
        hipLaunchKernelGGL(k_reparam<SV_F32>, dim3(blocks), dim3(256), 0, s, ml, eps, npix, L, (float *)z);
        break;
    case SV_BF16:
        hipLaunchKernelGGL(k_reparam<SV_BF16>, dim3(blocks), dim3(256), 0, s, ml, eps, npix, L, (uint16_t *)z);
        break;
    case SV_F16:
        hipLaunchKernelGGL(k_reparam<SV_F16>, dim3(blocks), dim3(256), 0, s, ml, eps, npix, L, (uint16_t *)z);
        break;
    default:
        return SV_ERR_DTYPE;
    }
    SV_LAUNCH_CHECK("k_reparam");
    return SV_OK;
}

}  // namespace sv
