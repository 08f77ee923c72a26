// Coarse matching kernels: block-mean reduction + census transform, and
// Hamming cost + winner-take-all with the disparity sweep held in registers.
//
// Census is named but not defined in the paper (Sec. I, Sec. III, variants S1/S2
// of Sec. IV-C); the definition used is the usual one: a bit per window
// neighbour, set when the neighbour is strictly darker than the centre.
// Winner-take-all is Eq. (6) on the raw (unaggregated) Hamming cost.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace sv {

// ---------------------------------------------------------------------------
// Reduction + census.  One workgroup (256 threads) = CEN_TW x TH reduced pixels
// of one image, TH = 4 or 16 (taller tiles re-read less halo; shorter ones
// give more workgroups for a single small frame).  The reduced patch with its
// clamped halo is built once in LDS (each patch pixel is the block mean of
// F x F full-resolution bytes: for F = 2, 4 four patch pixels per lane from
// one vector load per full-resolution row, else byte loads of several pixels
// unrolled and in flight together), then every thread packs the census words
// of its pixels from LDS.
// ---------------------------------------------------------------------------
constexpr int CEN_TW = CEN_TILE_W, CEN_MAXR = 8;
constexpr int CEN_THREADS = 256;
template <int TH>
using CenPatch = uint8_t[TH + 2 * CEN_MAXR][CEN_TW + 2 * CEN_MAXR];

// The census word of the pixel at patch (py, px): bit k for the k-th window
// neighbour (rows dy = -ry..ry outer, columns dx = -rx..rx inner, the centre
// skipped) strictly darker than the centre.  RX, RY > 0: the window is a
// compile-time constant and the loop is unrolled into byte reads at fixed LDS
// offsets; RX = RY = 0: the window is read from rx, ry at run time.
template <int TH, int RX, int RY>
__device__ __forceinline__ uint64_t census_word(const CenPatch<TH> &patch, int py, int px, int rx, int ry) {
    const uint32_t c = patch[py][px];
    if constexpr (RX > 0) {
        uint32_t lo = 0, hi = 0;
        int k = 0;
#pragma unroll
        for (int dy = -RY; dy <= RY; ++dy)
#pragma unroll
            for (int dx = -RX; dx <= RX; ++dx) {
                if (dy == 0 && dx == 0) continue;
                // (v - c) wraps to a value with the top bit set exactly when v < c
                const uint32_t bit = ((uint32_t)patch[py + dy][px + dx] - c) >> 31;
                if (k < 32) lo |= bit << k;
                else hi |= bit << (k - 32);
                ++k;
            }
        return ((uint64_t)hi << 32) | lo;
    } else {
        uint64_t code = 0;
        int k = 0;
        for (int dy = -ry; dy <= ry; ++dy)
            for (int dx = -rx; dx <= rx; ++dx) {
                if (dy == 0 && dx == 0) continue;
                code |= (uint64_t)(patch[py + dy][px + dx] < c) << k;
                ++k;
            }
        return code;
    }
}

// The census words of the four pixels at patch (py, c0 + RX .. c0 + RX + 3)
// for a compile-time window, the patch a byte array with rows of `stride`
// bytes (both the array and stride 4-byte aligned, c0 a multiple of 4):
// every window row is read once as the aligned words that hold columns
// c0 .. c0 + 3 + 2 RX, and the bytes are taken from registers.  Bit order and
// comparison as in census_word.
template <int RX, int RY>
__device__ __forceinline__ void census_words4_p(const uint8_t *patch, int stride, int py, int c0,
                                                uint64_t code[4]) {
    constexpr int NW = (4 + 2 * RX + 3) / 4, NR = 2 * RY + 1;
    uint32_t row[NR][NW];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < NW; ++k)
            row[r][k] = *(const uint32_t *)(patch + (size_t)(py - RY + r) * stride + c0 + 4 * k);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const uint32_t c = (row[RY][(g + RX) >> 2] >> (8 * ((g + RX) & 3))) & 0xffu;
        uint32_t lo = 0, hi = 0;
        int k = 0;
#pragma unroll
        for (int dy = -RY; dy <= RY; ++dy)
#pragma unroll
            for (int dx = -RX; dx <= RX; ++dx) {
                if (dy == 0 && dx == 0) continue;
                const int col = g + RX + dx;
                const uint32_t v = (row[dy + RY][col >> 2] >> (8 * (col & 3))) & 0xffu;
                const uint32_t bit = (v - c) >> 31;
                if (k < 32) lo |= bit << k;
                else hi |= bit << (k - 32);
                ++k;
            }
        code[g] = ((uint64_t)hi << 32) | lo;
    }
}

template <int TH, int RX, int RY>
__device__ __forceinline__ void census_words4(const CenPatch<TH> &patch, int py, int c0, uint64_t code[4]) {
    census_words4_p<RX, RY>(&patch[0][0], CEN_TW + 2 * CEN_MAXR, py, c0, code);
}

// The block mean of reduced pixel (i, j), clamped into the reduced image; a
// block cut by the image edge averages the bytes it holds (round half up).
// Every load is issued before the sum (a row or column past the edge re-reads
// the block's first byte and is left out).
template <int F>
__device__ __forceinline__ uint32_t block_mean(const uint8_t *__restrict__ img, int H, int W, int pitch,
                                               int h, int w, int i, int j) {
    i = min(max(i, 0), h - 1);
    j = min(max(j, 0), w - 1);
    const int ny = min(F, H - F * i), nx = min(F, W - F * j);
    const uint8_t *src = img + (size_t)(F * i) * pitch + F * j;
    uint32_t v[F * F];
#pragma unroll
    for (int y = 0; y < F; ++y)
#pragma unroll
        for (int x = 0; x < F; ++x) v[y * F + x] = src[(y < ny ? (size_t)y * pitch : 0) + (x < nx ? x : 0)];
    uint32_t sum = 0;
#pragma unroll
    for (int y = 0; y < F; ++y)
#pragma unroll
        for (int x = 0; x < F; ++x) sum += (y < ny && x < nx) ? v[y * F + x] : 0u;
    const uint32_t n = (uint32_t)(ny * nx);
    return (sum + n / 2) / n;
}

// The reduced patch of a tile for F = 2 or 4 and a compile-time window: a lane
// builds four horizontally adjacent patch pixels from F full-resolution rows,
// one vector load of 4F bytes per row (the rows of an image of odd pitch are
// not 4-byte aligned: these loads rely on the unaligned global access the
// GPU runs in), summed with v_sad_u8 and stored to LDS as one word.  Groups
// that reach a clamped or edge-cut block take the per-pixel path.
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t u32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));

template <int F, int TH, int RX, int RY>
__device__ __forceinline__ void reduce_patch4(CenPatch<TH> &patch, const uint8_t *__restrict__ img, int H,
                                              int W, int pitch, int h, int w, int i0, int j0) {
    static_assert(F == 2 || F == 4, "vector path for F = 2, 4");
    constexpr int PH = TH + 2 * RY, PW = CEN_TW + 2 * RX, NG = (PW + 3) / 4;
    static_assert(4 * NG <= CEN_TW + 2 * CEN_MAXR, "groups fit the patch row");
    // groups per thread, all of whose loads are issued before any is summed
    constexpr int NI = (PH * NG + CEN_THREADS - 1) / CEN_THREADS;
    using V = typename std::conditional<F == 4, u32x4_a4, u32x2_a4>::type;
    const int hc = H / F, wc = W / F;  // whole blocks
    V v[NI][F];
    bool fast[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int e = threadIdx.x + k * CEN_THREADS;
        const int pr = e / NG, cg = e - pr * NG;
        const int i = i0 + pr - RY, jg = j0 - RX + 4 * cg;
        fast[k] = e < PH * NG && i >= 0 && i < hc && jg >= 0 && jg + 3 < wc;
        if (fast[k]) {
            const uint8_t *src = img + (size_t)(F * i) * pitch + F * jg;
#pragma unroll
            for (int y = 0; y < F; ++y) v[k][y] = *(const V *)(src + (size_t)y * pitch);
        }
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int e = threadIdx.x + k * CEN_THREADS;
        if (e >= PH * NG) break;
        const int pr = e / NG, cg = e - pr * NG;
        uint32_t word;
        if (fast[k]) {
            uint32_t s0 = F * F / 2, s1 = s0, s2 = s0, s3 = s0;
#pragma unroll
            for (int y = 0; y < F; ++y) {
                if constexpr (F == 4) {
                    s0 = __builtin_amdgcn_sad_u8(v[k][y][0], 0u, s0);
                    s1 = __builtin_amdgcn_sad_u8(v[k][y][1], 0u, s1);
                    s2 = __builtin_amdgcn_sad_u8(v[k][y][2], 0u, s2);
                    s3 = __builtin_amdgcn_sad_u8(v[k][y][3], 0u, s3);
                } else {
                    s0 = __builtin_amdgcn_sad_u8(v[k][y][0] & 0xffffu, 0u, s0);
                    s1 = __builtin_amdgcn_sad_u8(v[k][y][0] >> 16, 0u, s1);
                    s2 = __builtin_amdgcn_sad_u8(v[k][y][1] & 0xffffu, 0u, s2);
                    s3 = __builtin_amdgcn_sad_u8(v[k][y][1] >> 16, 0u, s3);
                }
            }
            constexpr int SH = F == 4 ? 4 : 2;  // / (F * F)
            word = (s0 >> SH) | ((s1 >> SH) << 8) | ((s2 >> SH) << 16) | ((s3 >> SH) << 24);
        } else {
            const int i = i0 + pr - RY, jg = j0 - RX + 4 * cg;
            word = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                word |= block_mean<F>(img, H, W, pitch, h, w, i, jg + q) << (8 * q);
        }
        *(uint32_t *)&patch[pr][4 * cg] = word;
    }
}

// The reduced patch of a tile, any F and window: a thread reads the F x F
// bytes of several patch pixels (F is a template parameter so that the loads
// of R pixels are unrolled and in flight together) before summing any.
template <int F, int TH>
__device__ __forceinline__ void reduce_patch(CenPatch<TH> &patch, const uint8_t *__restrict__ img, int H,
                                             int W, int pitch, int rx, int ry, int h, int w, int i0, int j0) {
    constexpr int R = F * F >= 48 ? 1 : (48 / (F * F) > 4 ? 4 : 48 / (F * F));
    const int PH = TH + 2 * ry, PW = CEN_TW + 2 * rx;
    const int tid = threadIdx.x;
    for (int e0 = 0; e0 < PH * PW; e0 += R * CEN_THREADS) {
        uint32_t v[R][F * F];
        int ny[R], nx[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int e = e0 + k * CEN_THREADS + tid;
            const int ee = e < PH * PW ? e : 0;
            const int py = ee / PW, px = ee - py * PW;
            const int i = min(max(i0 + py - ry, 0), h - 1);
            const int j = min(max(j0 + px - rx, 0), w - 1);
            ny[k] = min(F, H - F * i);
            nx[k] = min(F, W - F * j);
            const uint8_t *src = img + (size_t)(F * i) * pitch + F * j;
#pragma unroll
            for (int y = 0; y < F; ++y)
#pragma unroll
                for (int x = 0; x < F; ++x)
                    // a row or column past the image edge re-reads the block's
                    // first byte and is dropped from the sum below
                    v[k][y * F + x] = src[(y < ny[k] ? (size_t)y * pitch : 0) + (x < nx[k] ? x : 0)];
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int e = e0 + k * CEN_THREADS + tid;
            if (e >= PH * PW) continue;
            uint32_t sum = 0;
#pragma unroll
            for (int y = 0; y < F; ++y)
#pragma unroll
                for (int x = 0; x < F; ++x)
                    sum += (y < ny[k] && x < nx[k]) ? v[k][y * F + x] : 0u;
            const int py = e / PW, px = e - py * PW;
            const uint32_t n = (uint32_t)(ny[k] * nx[k]);
            patch[py][px] = (uint8_t)(n == F * F ? (sum + F * F / 2) / (F * F) : (sum + n / 2) / n);
        }
    }
}

// One tile of one image: img is that image ([H][pitch]), low/cen its [h][w] maps.
// The reduced patch with its clamped halo is built in LDS, then every thread
// packs the census words of its pixels from LDS.
template <int F, int TH, int RX = 0, int RY = 0>
__device__ __forceinline__ void census_tile(CenPatch<TH> &patch, const uint8_t *__restrict__ img,
                                            int H, int W, int pitch, int rx, int ry, int h, int w,
                                            int i0, int j0, uint8_t *__restrict__ low,
                                            uint64_t *__restrict__ cen)
{
    if constexpr (RX > 0) {
        rx = RX;
        ry = RY;
    }
    if constexpr (RX > 0 && (F == 2 || F == 4))
        reduce_patch4<F, TH, RX, RY>(patch, img, H, W, pitch, h, w, i0, j0);
    else
        reduce_patch<F, TH>(patch, img, H, W, pitch, rx, ry, h, w, i0, j0);
    const int tid = threadIdx.x;
    __syncthreads();
    if constexpr (RX > 0 && TH >= 16) {
        // four horizontally adjacent pixels per thread, from aligned words
        // (short tiles keep one pixel per thread: all four waves busy)
        constexpr int NQ = CEN_TW / 4;
        const int q = tid % NQ, jq = j0 + 4 * q;
        for (int ty = tid / NQ; ty < TH; ty += CEN_THREADS / NQ) {
            const int i = i0 + ty;
            if (i >= h || jq >= w) continue;
            uint64_t code[4];
            census_words4<TH, RX, RY>(patch, ty + RY, 4 * q, code);
            const size_t o = (size_t)i * w + jq;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                if (jq + g < w) {
                    cen[o + g] = code[g];
                    if (low) low[o + g] = patch[ty + RY][4 * q + g + RX];
                }
            }
        }
    } else {
        const int tx = tid % CEN_TW;
        for (int ty = tid / CEN_TW; ty < TH; ty += CEN_THREADS / CEN_TW) {
            const int i = i0 + ty, j = j0 + tx;
            if (i < h && j < w) {
                const uint64_t code = census_word<TH, RX, RY>(patch, ty + ry, tx + rx, rx, ry);
                const size_t o = (size_t)i * w + j;
                cen[o] = code;
                if (low) low[o] = patch[ty + ry][tx + rx];
            }
        }
    }
    __syncthreads();  // the patch is reused by the next tile of a persistent loop
}

template <int F, int TH, int RX = 0, int RY = 0>
__global__ void __launch_bounds__(CEN_THREADS)
k_reduce_census(const uint8_t *__restrict__ img0, const uint8_t *__restrict__ img1, int B, int H,
                int W, int pitch, int rx, int ry, int h, int w, uint8_t *__restrict__ low0,
                uint8_t *__restrict__ low1, uint64_t *__restrict__ cen0,
                uint64_t *__restrict__ cen1)
{
    __shared__ __attribute__((aligned(16))) CenPatch<TH> patch;
    // z = image x view (one view when img1 is NULL)
    const int nv = img1 ? 2 : 1;
    const int view = blockIdx.z % nv;
    const int b = blockIdx.z / nv;
    const uint8_t *img = (view ? img1 : img0) + (size_t)b * H * pitch;
    uint8_t *low = view ? low1 : low0;
    uint64_t *cen = (view ? cen1 : cen0) + (size_t)b * h * w;
    census_tile<F, TH, RX, RY>(patch, img, H, W, pitch, rx, ry, h, w, blockIdx.y * TH, blockIdx.x * CEN_TW,
                               low ? low + (size_t)b * h * w : nullptr, cen);
}

#define SV_FACTOR_SWITCH(f, CALL) \
    switch (f) {                  \
    case 1: CALL(1); break;       \
    case 2: CALL(2); break;       \
    case 3: CALL(3); break;       \
    case 4: CALL(4); break;       \
    case 5: CALL(5); break;       \
    case 6: CALL(6); break;       \
    case 7: CALL(7); break;       \
    case 8: CALL(8); break;       \
    default: return SV_ERR_RANGE; \
    }

// Tall tiles once they still give two workgroups per CU.
int census_tile_height(int B, int h, int w) {
    const long long tall = 2LL * B * cdiv(w, CEN_TW) * cdiv(h, 16);
    return tall >= 512 ? 16 : 4;
}

sv_status launch_reduce_census(const uint8_t *img0, const uint8_t *img1, int B, int H, int W,
                               int pitch, int f, int win_w, int win_h, uint8_t *low0,
                               uint8_t *low1, uint64_t *cen0, uint64_t *cen1, hipStream_t s)
{
    const int h = cdiv(H, f), w = cdiv(W, f);
    const int th = census_tile_height(B, h, w);
    dim3 grid(cdiv(w, CEN_TW), cdiv(h, th), (img1 ? 2 : 1) * B);
    const int rx = (win_w - 1) / 2, ry = (win_h - 1) / 2;
#define SV_CEN_L(F, TH, RX, RY)                                                                    \
    hipLaunchKernelGGL((k_reduce_census<F, TH, RX, RY>), grid, dim3(CEN_THREADS), 0, s, img0, img1, \
                       B, H, W, pitch, rx, ry, h, w, low0, low1, cen0, cen1)
#define SV_CEN_W(F, TH)                                                                            \
    if (rx == 4 && ry == 3) SV_CEN_L(F, TH, 4, 3);                                                 \
    else if (rx == 2 && ry == 2) SV_CEN_L(F, TH, 2, 2);                                            \
    else SV_CEN_L(F, TH, 0, 0)
#define SV_CEN_LAUNCH(F)                                                                           \
    if (F != 2 && F != 4) {                                                                        \
        if (th == 16) SV_CEN_L(F, 16, 0, 0); else SV_CEN_L(F, 4, 0, 0);                            \
    } else if (th == 16) {                                                                         \
        SV_CEN_W(F, 16);                                                                           \
    } else {                                                                                       \
        SV_CEN_W(F, 4);                                                                            \
    }
    SV_FACTOR_SWITCH(f, SV_CEN_LAUNCH)
#undef SV_CEN_LAUNCH
#undef SV_CEN_W
#undef SV_CEN_L
    SV_LAUNCH_CHECK("k_reduce_census");
    return SV_OK;
}

// Persistent variant: tiles of both views of every pair of the table; the
// per-pair maps live in flattened buffers at the pair's level-0 offset.
template <int F, int TH, int RX = 0, int RY = 0>
__global__ void __launch_bounds__(CEN_THREADS)
k_reduce_census_tab(const PairTable *__restrict__ tab, int rx, int ry, uint8_t *__restrict__ low0,
                    uint64_t *__restrict__ cen0, uint64_t *__restrict__ cen1)
{
    __shared__ __attribute__((aligned(16))) CenPatch<TH> patch;
    const int n = tab->n;
    const int *cum = tab->cum[BS_CENSUS];
    const int total = cum[n];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = table_find(cum, n, t);
        const PairGeo &g = tab->pair[i];
        const int local = t - cum[i];
        const int tw = cdiv_d(g.w[0], CEN_TW), th = cdiv_d(g.h[0], TH);
        const int view = local / (tw * th), r = local - view * tw * th;
        const long long o = g.off[0];
        census_tile<F, TH, RX, RY>(patch, view ? g.right : g.left, g.H, g.W, g.W, rx, ry, g.h[0], g.w[0],
                           (r / tw) * TH, (r % tw) * CEN_TW, view ? nullptr : low0 + o,
                           (view ? cen1 : cen0) + o);
    }
}

sv_status launch_reduce_census_tab(const PairTable *tab, int grid, int f, int th, int win_w,
                                   int win_h, uint8_t *low0, uint64_t *cen0, uint64_t *cen1,
                                   hipStream_t s)
{
    if (th != 4 && th != 16) return SV_ERR_RANGE;
    const int rx = (win_w - 1) / 2, ry = (win_h - 1) / 2;
#define SV_CEN_L(F, TH, RX, RY)                                                                    \
    hipLaunchKernelGGL((k_reduce_census_tab<F, TH, RX, RY>),                                       \
                       dim3((unsigned)resident_grid((const void *)k_reduce_census_tab<F, TH, RX, RY>, 0, grid)), \
                       dim3(CEN_THREADS), 0, s, tab, rx, ry, low0, cen0, cen1)
#define SV_CEN_W(F, TH)                                                                            \
    if (rx == 4 && ry == 3) SV_CEN_L(F, TH, 4, 3);                                                 \
    else if (rx == 2 && ry == 2) SV_CEN_L(F, TH, 2, 2);                                            \
    else SV_CEN_L(F, TH, 0, 0)
#define SV_CEN_LAUNCH(F)                                                                           \
    if (F != 2 && F != 4) {                                                                        \
        if (th == 16) SV_CEN_L(F, 16, 0, 0); else SV_CEN_L(F, 4, 0, 0);                            \
    } else if (th == 16) {                                                                         \
        SV_CEN_W(F, 16);                                                                           \
    } else {                                                                                       \
        SV_CEN_W(F, 4);                                                                            \
    }
    SV_FACTOR_SWITCH(f, SV_CEN_LAUNCH)
#undef SV_CEN_LAUNCH
#undef SV_CEN_W
#undef SV_CEN_L
    SV_LAUNCH_CHECK("k_reduce_census_tab");
    return SV_OK;
}

// ---------------------------------------------------------------------------
// Hamming cost + WTA.  One workgroup = one row segment of CW_TW pixels; each
// pixel is served by DSPLIT adjacent lanes that sweep d = k, k + DSPLIT, ...
// in registers, keeping the packed key (cost << 8) | d; an unsigned min over
// keys picks the least cost and, among equal costs, the lowest d, in any
// reduction order.  The right census row segment [j0 - D + 1, j0 + CW_TW) is
// staged once in LDS.  The lanes of one pixel then combine keys by shuffle.
// ---------------------------------------------------------------------------
constexpr int CW_THREADS = 256;
int cost_wta_tile_width(int dsplit) { return CW_THREADS / dsplit; }

// One row segment [j0, j0 + TW) of one row (cl, cr, disp point at the row).
template <int DSPLIT>
__device__ __forceinline__ void cost_wta_seg(uint64_t *rseg, const uint64_t *__restrict__ cl,
                                             const uint64_t *__restrict__ cr, int w, int D,
                                             int nbits, uint8_t *__restrict__ disp,
                                             uint8_t *__restrict__ disp2, int j0)
{
    constexpr int TW = CW_THREADS / DSPLIT;
    const int base = j0 - (D - 1);  // column of rseg[0]
    for (int e = threadIdx.x; e < TW + D - 1; e += CW_THREADS) {
        const int x = base + e;
        rseg[e] = (x >= 0 && x < w) ? cr[x] : 0;
    }
    __syncthreads();
    const int p = threadIdx.x / DSPLIT, k = threadIdx.x % DSPLIT;
    const int j = j0 + p;
    const uint64_t lv = (j < w) ? cl[j] : 0;
    uint32_t best = 0xffffffffu;
    // d <= j compares with column j - d, which sits at rseg[p + D - 1 - d];
    // every d > j costs the sentinel, so of those only the lowest of this
    // lane's sequence k, k + DSPLIT, ... can win
    const int dend = min(D, j + 1);
    const uint64_t *rp = rseg + p + D - 1;
#pragma unroll 4
    for (int d = k; d < dend; d += DSPLIT)
        best = min(best, ((uint32_t)__popcll(lv ^ rp[-d]) << 8) | (uint32_t)d);
    const int dfirst = k + DSPLIT * ((max(dend - k, 0) + DSPLIT - 1) / DSPLIT);
    if (dfirst < D) best = min(best, ((uint32_t)(nbits + 1) << 8) | (uint32_t)dfirst);
#pragma unroll
    for (int m = 1; m < DSPLIT; m <<= 1) best = min(best, (uint32_t)__shfl_xor((int)best, m));
    if (k == 0 && j < w) {
        disp[j] = (uint8_t)(best & 0xffu);
        if (disp2) disp2[j] = (uint8_t)(best & 0xffu);
    }
    __syncthreads();
}

// A workgroup takes rows blockIdx.y * rpw .. + rpw - 1 of its column segment
// (several rows per workgroup at large batch: short-lived workgroups cost more
// to launch than they compute).
template <int DSPLIT>
__global__ void __launch_bounds__(CW_THREADS)
k_cost_wta(const uint64_t *__restrict__ cl, const uint64_t *__restrict__ cr, int h, int w, int D,
           int nbits, int rpw, uint8_t *__restrict__ disp)
{
    __shared__ uint64_t rseg[CW_THREADS / DSPLIT + 256];
    const int r1 = min(h, (int)(blockIdx.y + 1) * rpw);
    for (int r = blockIdx.y * rpw; r < r1; ++r) {
        const size_t row = ((size_t)blockIdx.z * h + r) * w;
        cost_wta_seg<DSPLIT>(rseg, cl + row, cr + row, w, D, nbits, disp + row, nullptr,
                             blockIdx.x * (CW_THREADS / DSPLIT));
    }
}

template <int DSPLIT>
__global__ void __launch_bounds__(CW_THREADS)
k_cost_wta_tab(const PairTable *__restrict__ tab, const uint64_t *__restrict__ cl,
               const uint64_t *__restrict__ cr, int nbits, uint8_t *__restrict__ disp)
{
    constexpr int TW = CW_THREADS / DSPLIT;
    __shared__ uint64_t rseg[TW + 256];
    const int n = tab->n;
    const int *cum = tab->cum[BS_COST_WTA];
    const int total = cum[n];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = table_find(cum, n, t);
        const PairGeo &g = tab->pair[i];
        const int local = t - cum[i];
        const int segs = cdiv_d(g.w[0], TW);
        const int r = local / segs, j0 = (local % segs) * TW;
        const size_t row = (size_t)g.off[0] + (size_t)r * g.w[0];
        cost_wta_seg<DSPLIT>(rseg, cl + row, cr + row, g.w[0], g.D, nbits, disp + row,
                             g.disp_out ? g.disp_out + (size_t)r * g.w[0] : nullptr, j0);
    }
}

sv_status launch_cost_wta_tab(const PairTable *tab, int grid, const uint64_t *cl, const uint64_t *cr,
                              int nbits, uint8_t *disp, int dsplit, hipStream_t s)
{
    switch (dsplit) {
#define SV_CWT_CASE(N)                                                                             \
    case N:                                                                                        \
        hipLaunchKernelGGL(k_cost_wta_tab<N>, dim3((unsigned)resident_grid((const void *)k_cost_wta_tab<N>, 0, grid)), \
                           dim3(CW_THREADS), 0, s, tab, cl, cr, nbits, disp);                      \
        break;
        SV_CWT_CASE(1)
        SV_CWT_CASE(2)
        SV_CWT_CASE(4)
        SV_CWT_CASE(8)
#undef SV_CWT_CASE
    default:
        return SV_ERR_RANGE;
    }
    SV_LAUNCH_CHECK("k_cost_wta_tab");
    return SV_OK;
}

sv_status launch_cost_wta(const uint64_t *cl, const uint64_t *cr, int B, int h, int w, int D,
                          int nbits, uint8_t *disp, int dsplit, hipStream_t s)
{
    // rows per workgroup: 4 once that still leaves 8 workgroups per CU
    const long long wgs = (long long)cdiv(w, CW_THREADS / dsplit) * h * B;
    const int rpw = wgs >= 4 * 2048 ? 4 : 1;
    switch (dsplit) {
#define SV_CW_CASE(N)                                                                      \
    case N: {                                                                              \
        dim3 grid(cdiv(w, CW_THREADS / N), cdiv(h, rpw), B);                               \
        hipLaunchKernelGGL(k_cost_wta<N>, grid, dim3(CW_THREADS), 0, s, cl, cr, h, w, D,   \
                           nbits, rpw, disp);                                              \
        break;                                                                             \
    }
        SV_CW_CASE(1)
        SV_CW_CASE(2)
        SV_CW_CASE(4)
        SV_CW_CASE(8)
#undef SV_CW_CASE
    default:
        return SV_ERR_RANGE;
    }
    SV_LAUNCH_CHECK("k_cost_wta");
    return SV_OK;
}

}  // namespace sv
