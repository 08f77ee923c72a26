// Semi-global matching on the census cost (Sec. III-A2, Eqs. (4)-(5)), winner-
// take-all on the aggregated cost (Eq. (6)), the single matching phase
// (Sec. III-A3, Eq. (7)) and a 3 x 3 median filter: the Census + SGM member
// of the paper's matching family (S2 of Sec. IV-C), at the reduced
// resolution.
//
// The matching cost is first written as a uint8 volume.  Path costs (Eq. (4))
// run along the four axis directions: one 16-lane DPP row of a wavefront
// follows one path (four paths per wave); lane l holds the
// disparities d = l * DPL + j, j < DPL, in registers, so d - 1 and d + 1 are
// in the same lane except at the ends of its run, which come from the
// neighbouring lanes by DPP row shifts, and min_k C_r(p - r, k) is a DPP row
// rotate-and-min.  Each direction writes its path costs C_r as uint8 into a
// volume of its own, and the WTA kernel sums the four (Eq. (5)).
#include "common.h"
#include "kernels.h"

namespace sv {

constexpr int SGM_INF = 0x3fff;        // above any path cost (uint8 range)
constexpr int SGM_LANES = 16;          // lanes per path = one DPP row

template <int CTRL>
__device__ __forceinline__ int dpp(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xf, 0xf, false);
}
// min over the 16 lanes of a DPP row, in every lane of the row
__device__ __forceinline__ int row_min(int v) {
    v = min(v, dpp<0x121>(0, v));  // row_ror:1
    v = min(v, dpp<0x122>(0, v));  // row_ror:2
    v = min(v, dpp<0x124>(0, v));  // row_ror:4
    v = min(v, dpp<0x128>(0, v));  // row_ror:8
    return v;
}

// Matching cost volume C(p, d) (the cost of Eq. (6): Hamming distance of the
// census codes, nbits + 1 where x - d < 0) as uint8 [B][h][w][Dp], Dp = D
// rounded up to a multiple of 4 (the padding is never read as a cost).  One
// workgroup = a row segment of CV_TW pixels; the right census codes it needs,
// [j0 - D + 1, j0 + CV_TW), are staged in LDS once; a thread writes four
// disparities of a pixel as one 32-bit word.
constexpr int CV_TW = 64;
__global__ void __launch_bounds__(256)
k_sgm_cost(const uint64_t *__restrict__ cl, const uint64_t *__restrict__ cr, int h, int w, int D,
           int Dp, int nbits, uint8_t *__restrict__ cost)
{
    __shared__ uint64_t seg[CV_TW + 256];
    const size_t row = ((size_t)blockIdx.z * h + blockIdx.y) * w;
    const int j0 = blockIdx.x * CV_TW;
    const int base = j0 - (D - 1);
    for (int e = threadIdx.x; e < CV_TW + D - 1; e += blockDim.x) {
        const int x = base + e;
        seg[e] = (x >= 0 && x < w) ? cr[row + x] : 0;
    }
    __syncthreads();
    const int ng = Dp / 4;
    for (int e = threadIdx.x; e < CV_TW * ng; e += blockDim.x) {
        const int px = e / ng, g = e - px * ng;
        const int j = j0 + px;
        if (j >= w) continue;
        const uint64_t lv = cl[row + j];
        uint32_t word = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int d = 4 * g + k;
            // column j - d of the right view is seg[px + D - 1 - d]
            const uint32_t c = d >= D ? 0u
                             : (j - d < 0 ? (uint32_t)(nbits + 1)
                                          : (uint32_t)__popcll(lv ^ seg[px + D - 1 - (d < D ? d : 0)]));
            word |= c << (8 * k);
        }
        *(uint32_t *)(cost + (row + j) * Dp + 4 * g) = word;
    }
}

// Path p of npath: directions 0 (left to right) and 1 (right to left) run
// along rows, 2 (top to bottom) and 3 (bottom to top) along columns;
// vol[dir][b][y][x][Dp].  The step's costs are loaded SGM_PF steps ahead into
// a ring of registers, so the dependent chain of a step is arithmetic and DPP
// only.
constexpr int SGM_PF = 16;
template <int DPL>
struct CostWords {
    static constexpr int N = DPL >= 4 ? DPL / 4 : 1;
    uint32_t v[N];
    uint32_t ok;  // bit k: word k holds costs (else it is read as zero)
};

// The costs of disparities d0 .. d0 + DPL - 1 of one pixel (p points at d0).
// The loads are unconditional (a word at or past Dp, or of a step past the
// path's end, reads `safe` instead) and the mask is applied where the costs
// are used, so nothing waits for a load until its step comes.
template <int DPL>
__device__ __forceinline__ void load_costs(const uint8_t *__restrict__ p, const uint8_t *safe, bool ok,
                                           int d0, int Dp, CostWords<DPL> &c) {
    c.ok = 0;
    if constexpr (DPL >= 4) {
#pragma unroll
        for (int k = 0; k < DPL / 4; ++k) {
            const bool okk = ok && d0 + 4 * k < Dp;
            c.v[k] = *(const uint32_t *)(okk ? p + 4 * k : safe);
            c.ok |= (uint32_t)okk << k;
        }
    } else if constexpr (DPL == 2) {
        c.v[0] = *(const uint16_t *)(ok ? p : safe);
        c.ok = ok;
    } else {
        c.v[0] = *(ok ? p : safe);
        c.ok = ok;
    }
}

template <int DPL>
__global__ void __launch_bounds__(64)
k_sgm_paths(const uint8_t *__restrict__ cost, int B, int h, int w, int D, int Dp, int P1, int P2,
            uint8_t *__restrict__ vol, uint8_t *__restrict__ sink)
{
    const int lane = threadIdx.x & (SGM_LANES - 1);
    const int path = blockIdx.x * 4 + (threadIdx.x >> 4);
    const int nrow = B * h, ncol = B * w;
    const int npath = 2 * nrow + 2 * ncol;
    if (path >= npath) return;  // whole DPP rows leave together
    int dir, line;
    if (path < 2 * nrow) { dir = path / nrow; line = path - dir * nrow; }
    else { const int q = path - 2 * nrow; dir = 2 + q / ncol; line = q - (dir - 2) * ncol; }
    int b, x0, y0, dx, dy, len;
    if (dir < 2) {
        b = line / h; y0 = line - b * h;
        dx = dir == 0 ? 1 : -1; dy = 0;
        x0 = dir == 0 ? 0 : w - 1;
        len = w;
    } else {
        b = line / w; x0 = line - b * w;
        dx = 0; dy = dir == 2 ? 1 : -1;
        y0 = dir == 2 ? 0 : h - 1;
        len = h;
    }
    const size_t plane = (size_t)h * w;
    const uint8_t *cb = cost + (size_t)b * plane * Dp;
    uint8_t *vb = vol + ((size_t)dir * B + b) * plane * Dp;
    const int d0 = lane * DPL;
    const bool lane_ok = d0 < Dp;
    // pixel offset (in pixels) of step s
    const long long step_px = (long long)dy * w + dx;
    const long long px0 = (long long)y0 * w + x0;
    // words of lanes past Dp are stored to a per-lane sink (never read), so
    // stores, like loads, need no branch
    uint8_t *my_sink = sink + (size_t)(threadIdx.x & 63) * 64;

    CostWords<DPL> ring[SGM_PF];
#pragma unroll
    for (int k = 0; k < SGM_PF; ++k)
        load_costs<DPL>(cb + (size_t)(px0 + (long long)(k < len ? k : 0) * step_px) * Dp + d0, cb,
                        lane_ok && k < len, d0, Dp, ring[k]);

    int prev[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) prev[j] = SGM_INF;
    int mprev = 0;
    // one step s of the path, its costs in ring slot k (refilled with step s + SGM_PF)
    auto step = [&](int k, int s) {
        int c[DPL];
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const int q = DPL >= 4 ? j / 4 : 0;
            const uint32_t word = ((ring[k].ok >> q) & 1u) ? ring[k].v[q] : 0u;
            const int sh = DPL >= 4 ? 8 * (j % 4) : 8 * j;
            c[j] = d0 + j < D ? (int)((word >> sh) & 0xffu) : SGM_INF;
        }
        const int sn = s + SGM_PF;
        load_costs<DPL>(cb + (size_t)(px0 + (long long)(sn < len ? sn : 0) * step_px) * Dp + d0, cb,
                        lane_ok && sn < len, d0, Dp, ring[k]);
        int cur[DPL];
        if (s == 0) {
#pragma unroll
            for (int j = 0; j < DPL; ++j) cur[j] = c[j];
        } else {
            const int from_left = dpp<0x111>(SGM_INF, prev[DPL - 1]);  // row_shr:1: lane - 1
            const int from_right = dpp<0x101>(SGM_INF, prev[0]);       // row_shl:1: lane + 1
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                const int lft = j > 0 ? prev[j - 1] : from_left;
                const int rgt = j + 1 < DPL ? prev[j + 1] : from_right;
                int m = min(prev[j], min(lft, rgt) + P1);
                m = min(m, mprev + P2);
                cur[j] = c[j] >= SGM_INF ? SGM_INF : c[j] + m - mprev;
            }
        }
        int mn = cur[0];
#pragma unroll
        for (int j = 1; j < DPL; ++j) mn = min(mn, cur[j]);
        mprev = row_min(mn);
        uint8_t *o = vb + (size_t)(px0 + (long long)s * step_px) * Dp + d0;
        if constexpr (DPL >= 4) {
#pragma unroll
            for (int q = 0; q < DPL / 4; ++q) {
                uint32_t word = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) word |= (uint32_t)(cur[4 * q + t] & 0xff) << (8 * t);
                const bool okq = lane_ok && d0 + 4 * q < Dp;
                *(uint32_t *)(okq ? o + 4 * q : my_sink + 4 * q) = word;
            }
        } else if constexpr (DPL == 2) {
            *(uint16_t *)(lane_ok ? o : my_sink) = (uint16_t)((cur[0] & 0xff) | ((cur[1] & 0xff) << 8));
        } else {
            *(lane_ok ? o : my_sink) = (uint8_t)cur[0];
        }
#pragma unroll
        for (int j = 0; j < DPL; ++j) prev[j] = cur[j];
    };
    int s0 = 0;
    for (; s0 + SGM_PF <= len; s0 += SGM_PF) {
#pragma unroll
        for (int k = 0; k < SGM_PF; ++k) step(k, s0 + k);
    }
#pragma unroll
    for (int k = 0; k < SGM_PF; ++k)
        if (s0 + k < len) step(k, s0 + k);
}

// Aggregated cost (Eq. (5)) and winner-take-all (Eq. (6)), lowest d on ties;
// the four volumes are [B][h][w][Dp].
__global__ void __launch_bounds__(256)
k_sgm_wta(const uint8_t *__restrict__ vol, size_t nvox, int D, int Dp, size_t npix,
          uint8_t *__restrict__ disp)
{
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < npix;
         p += (size_t)gridDim.x * blockDim.x) {
        const uint8_t *v0 = vol + p * Dp, *v1 = v0 + nvox, *v2 = v1 + nvox, *v3 = v2 + nvox;
        int best = 0x7fffffff, bd = 0;
        for (int d = 0; d < D; d += 4) {
            const uint32_t a = *(const uint32_t *)(v0 + d), bq = *(const uint32_t *)(v1 + d);
            const uint32_t cq = *(const uint32_t *)(v2 + d), dq = *(const uint32_t *)(v3 + d);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int sh = 8 * k;
                const int s = (int)((a >> sh) & 0xff) + (int)((bq >> sh) & 0xff) +
                              (int)((cq >> sh) & 0xff) + (int)((dq >> sh) & 0xff);
                if (d + k < D && s < best) { best = s; bd = d + k; }
            }
        }
        disp[p] = (uint8_t)bd;
    }
}

// Single matching phase (Eq. (7)) with nearest-valid filling, one wave per
// row.  The target column of x is x - D(x); x is invalid when a pixel x + k,
// 0 < k < D, has the same target column (the left pixel of such a pair is
// the one hidden in the target view).  Validity is kept as one 64-bit ballot
// per 64 pixels; each invalid pixel takes the nearest valid value of its row
// (the smaller one at equal distances).  The row is staged in LDS.
constexpr int SMP_MAXW = 16384;
__global__ void __launch_bounds__(64)
k_smp(const uint8_t *__restrict__ disp, int B, int h, int w, int D, uint8_t *__restrict__ out)
{
    __shared__ uint8_t row[SMP_MAXW];
    __shared__ uint64_t valid[SMP_MAXW / 64];
    const int lane = threadIdx.x;
    const size_t base = (size_t)blockIdx.x * w;  // row blockIdx.x of B * h
    for (int x = lane; x < w; x += 64) row[x] = disp[base + x];
    __syncthreads();
    const int nch = (w + 63) / 64;
    for (int ch = 0; ch < nch; ++ch) {
        const int x = ch * 64 + lane;
        bool ok = x < w;
        if (ok) {
            const int t = x - row[x];
            for (int k = 1; k < D && x + k < w; ++k)
                if (x + k - row[x + k] == t) { ok = false; break; }
        }
        const uint64_t m = __ballot(ok);
        if (lane == 0) valid[ch] = m;
    }
    __syncthreads();
    bool any = false;
    for (int ch = 0; ch < nch; ++ch) any |= valid[ch] != 0;
    for (int x = lane; x < w; x += 64) {
        const int ch = x >> 6, bit = x & 63;
        uint8_t v = row[x];
        if (any && !((valid[ch] >> bit) & 1)) {
            // nearest valid index below x and above x (-1 / w when none)
            int lo = -1, hi = w;
            uint64_t mb = valid[ch] & ((bit ? (~0ull >> (64 - bit)) : 0ull));
            for (int c = ch; c >= 0; --c) {
                const uint64_t mm = c == ch ? mb : valid[c];
                if (mm) { lo = c * 64 + 63 - __clzll(mm); break; }
            }
            uint64_t ma = bit == 63 ? 0ull : valid[ch] & (~0ull << (bit + 1));
            for (int c = ch; c < nch; ++c) {
                const uint64_t mm = c == ch ? ma : valid[c];
                if (mm) { hi = c * 64 + __ffsll((unsigned long long)mm) - 1; break; }
            }
            const int dl = lo >= 0 ? x - lo : 0x7fffffff, dr = hi < w ? hi - x : 0x7fffffff;
            if (dl < dr) v = row[lo];
            else if (dr < dl) v = row[hi];
            else v = min(row[lo], row[hi]);
        }
        out[base + x] = v;
    }
}

// 3 x 3 median, borders replicated (median of nine by a fixed exchange network).
__device__ __forceinline__ void sort2(int &a, int &b) {
    const int t = min(a, b);
    b = max(a, b);
    a = t;
}
__global__ void __launch_bounds__(256)
k_median3(const uint8_t *__restrict__ in, int B, int h, int w, uint8_t *__restrict__ out)
{
    const size_t n = (size_t)B * h * w;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n;
         p += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(p % w);
        const size_t r = p / w;
        const int i = (int)(r % h);
        const uint8_t *img = in + (r - i) * w;
        const int ys[3] = {max(i - 1, 0), i, min(i + 1, h - 1)};
        const int xs[3] = {max(j - 1, 0), j, min(j + 1, w - 1)};
        int v[9];
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int t = 0; t < 3; ++t) v[u * 3 + t] = img[(size_t)ys[u] * w + xs[t]];
        // Paeth's 19-exchange median-of-nine network
        sort2(v[1], v[2]); sort2(v[4], v[5]); sort2(v[7], v[8]);
        sort2(v[0], v[1]); sort2(v[3], v[4]); sort2(v[6], v[7]);
        sort2(v[1], v[2]); sort2(v[4], v[5]); sort2(v[7], v[8]);
        sort2(v[0], v[3]); sort2(v[5], v[8]); sort2(v[4], v[7]);
        sort2(v[3], v[6]); sort2(v[1], v[4]); sort2(v[2], v[5]);
        sort2(v[4], v[7]); sort2(v[4], v[2]); sort2(v[6], v[4]);
        sort2(v[4], v[2]);
        out[p] = (uint8_t)v[4];
    }
}

static inline int sgm_dpad(int D) { return (D + 3) & ~3; }

// the cost volume, the four path-cost volumes, and a 4 KB sink for the
// stores of lanes past the padded disparity range
constexpr size_t SGM_SINK = 4096;
size_t sgm_volume_bytes(int B, int h, int w, int D) {
    return (size_t)5 * B * h * w * sgm_dpad(D) + SGM_SINK;
}

// Path sweeps + aggregation / WTA on a uint8 cost volume already in the
// workspace (ws: cost, four path volumes, sink).
static sv_status sgm_from_cost(int B, int h, int w, int D, int P1, int P2, uint8_t *ws, uint8_t *disp,
                               hipStream_t s)
{
    const int Dp = sgm_dpad(D);
    const size_t nvox = (size_t)B * h * w * Dp;
    const uint8_t *cost = ws;
    uint8_t *vol = ws + nvox, *sink = ws + 5 * nvox;
    const int npath = 2 * B * h + 2 * B * w;
    const dim3 grid(cdiv(npath, 4));
    const int dpl = cdiv(D, SGM_LANES);
#define SV_SGM(N) \
    hipLaunchKernelGGL(k_sgm_paths<N>, grid, dim3(64), 0, s, cost, B, h, w, D, Dp, P1, P2, vol, sink)
    if (dpl <= 1) SV_SGM(1);
    else if (dpl <= 2) SV_SGM(2);
    else if (dpl <= 4) SV_SGM(4);
    else if (dpl <= 8) SV_SGM(8);
    else SV_SGM(16);
#undef SV_SGM
    SV_LAUNCH_CHECK("k_sgm_paths");
    const size_t npix = (size_t)B * h * w;
    const int blocks = (int)std::min<size_t>((npix + 255) / 256, 8192);
    hipLaunchKernelGGL(k_sgm_wta, dim3(blocks), dim3(256), 0, s, vol, nvox, D, Dp, npix, disp);
    SV_LAUNCH_CHECK("k_sgm_wta");
    return SV_OK;
}

sv_status launch_sgm(const uint64_t *cl, const uint64_t *cr, int B, int h, int w, int D, int nbits,
                     int P1, int P2, uint8_t *ws, uint8_t *disp, hipStream_t s)
{
    const int Dp = sgm_dpad(D);
    hipLaunchKernelGGL(k_sgm_cost, dim3(cdiv(w, CV_TW), h, B), dim3(256), 0, s, cl, cr, h, w, D, Dp,
                       nbits, ws);
    SV_LAUNCH_CHECK("k_sgm_cost");
    return sgm_from_cost(B, h, w, D, P1, P2, ws, disp, s);
}

// ---------------------------------------------------------------------------
// Zero-mean normalised cross-correlation cost, Eqs. (1)-(3), on the reduced
// images.  With n window pixels (clamped to the image edge) and the exact
// integer window sums SR, SRR, ST, STT, SRT of the reference and target
// values,
//   C = 1 - N / sqrt(A B),  N = n SRT - SR ST,  A = n SRR - SR^2,  B = n STT - ST^2,
// evaluated in FP64 (C = 1 for a flat window, 2 where x - d < 0), and kept as
// q = floor(32 C + 1/2) in 0..64 for the path aggregation.  One workgroup =
// ZN_TW x ZN_TH pixels; the reference tile and the target tile (widened by
// D - 1 columns) with their window halos are staged in LDS; a thread holds its
// reference window in registers and runs over the disparities.
// ---------------------------------------------------------------------------
constexpr int ZN_TW = 64, ZN_TH = 4;

template <int RX, int RY>
__global__ void __launch_bounds__(ZN_TW * ZN_TH)
k_zncc_cost(const uint8_t *__restrict__ ll, const uint8_t *__restrict__ lr, int h, int w, int D,
            int Dp, uint8_t *__restrict__ cost)
{
    constexpr int PH = ZN_TH + 2 * RY, PWL = ZN_TW + 2 * RX;
    constexpr int NW = (2 * RX + 1) * (2 * RY + 1);
    __shared__ uint8_t pr[PH][PWL];
    __shared__ uint8_t pt[PH][ZN_TW + 2 * RX + 255];
    const int b = blockIdx.z;
    const int i0 = blockIdx.y * ZN_TH, j0 = blockIdx.x * ZN_TW;
    const uint8_t *L = ll + (size_t)b * h * w, *R = lr + (size_t)b * h * w;
    const int PWT = ZN_TW + 2 * RX + D - 1;  // target columns j0 - RX - (D - 1) ...
    for (int e = threadIdx.x; e < PH * PWL; e += blockDim.x) {
        const int py = e / PWL, px = e - py * PWL;
        const int y = min(max(i0 + py - RY, 0), h - 1), x = min(max(j0 + px - RX, 0), w - 1);
        pr[py][px] = L[(size_t)y * w + x];
    }
    for (int e = threadIdx.x; e < PH * PWT; e += blockDim.x) {
        const int py = e / PWT, px = e - py * PWT;
        const int y = min(max(i0 + py - RY, 0), h - 1);
        const int x = min(max(j0 - RX - (D - 1) + px, 0), w - 1);
        pt[py][px] = R[(size_t)y * w + x];
    }
    __syncthreads();
    const int ty = threadIdx.x / ZN_TW, tx = threadIdx.x - ty * ZN_TW;
    const int i = i0 + ty, j = j0 + tx;
    if (i >= h || j >= w) return;
    int rv[NW];
    int SR = 0, SRR = 0;
#pragma unroll
    for (int dy = 0; dy <= 2 * RY; ++dy)
#pragma unroll
        for (int dx = 0; dx <= 2 * RX; ++dx) {
            const int r = pr[ty + dy][tx + dx];
            rv[dy * (2 * RX + 1) + dx] = r;
            SR += r;
            SRR += r * r;
        }
    const long long n = NW;
    const long long A = n * SRR - (long long)SR * SR;
    uint8_t *o = cost + (((size_t)b * h + i) * w + j) * Dp;
    for (int d = 0; d < Dp; ++d) {
        int q = 0;
        if (d < D) {
            if (j - d < 0) {
                q = 64;
            } else {
                // target window of column j - d: pt column tx + dx + (D - 1) - d
                int ST = 0, STT = 0, SRT = 0;
#pragma unroll
                for (int dy = 0; dy <= 2 * RY; ++dy)
#pragma unroll
                    for (int dx = 0; dx <= 2 * RX; ++dx) {
                        const int t = pt[ty + dy][tx + dx + (D - 1) - d];
                        ST += t;
                        STT += t * t;
                        SRT += rv[dy * (2 * RX + 1) + dx] * t;
                    }
                const long long N = n * SRT - (long long)SR * ST;
                const long long Bv = n * STT - (long long)ST * ST;
                double C;
                if (A == 0 || Bv == 0) C = 1.0;
                else C = 1.0 - (double)N / sqrt((double)A * (double)Bv);
                q = (int)floor(32.0 * C + 0.5);
            }
        }
        o[d] = (uint8_t)q;
    }
}

bool zncc_window_supported(int win_w, int win_h) {
    const int rx = (win_w - 1) / 2, ry = (win_h - 1) / 2;
    if (win_w % 2 == 0 || win_h % 2 == 0) return false;
    return (rx == 1 && ry == 1) || (rx == 2 && ry == 2) || (rx == 3 && ry == 3) || (rx == 4 && ry == 3) ||
           (rx == 3 && ry == 4) || (rx == 4 && ry == 4) || (rx == 2 && ry == 1) || (rx == 1 && ry == 2);
}

sv_status launch_zncc_cost(const uint8_t *ll, const uint8_t *lr, int B, int h, int w, int D, int Dp,
                           int win_w, int win_h, uint8_t *cost, hipStream_t s)
{
    const dim3 grid(cdiv(w, ZN_TW), cdiv(h, ZN_TH), B);
    const int rx = (win_w - 1) / 2, ry = (win_h - 1) / 2;
#define SV_ZN(X, Y)                                                                                \
    if (rx == X && ry == Y) {                                                                      \
        hipLaunchKernelGGL((k_zncc_cost<X, Y>), grid, dim3(ZN_TW * ZN_TH), 0, s, ll, lr, h, w, D, Dp, \
                           cost);                                                                  \
        SV_LAUNCH_CHECK("k_zncc_cost");                                                            \
        return SV_OK;                                                                              \
    }
    SV_ZN(1, 1) SV_ZN(2, 2) SV_ZN(3, 3) SV_ZN(4, 3) SV_ZN(3, 4) SV_ZN(4, 4) SV_ZN(2, 1) SV_ZN(1, 2)
#undef SV_ZN
    return SV_ERR_UNSUPPORTED;
}

sv_status launch_zncc_sgm(const uint8_t *ll, const uint8_t *lr, int B, int h, int w, int D, int win_w,
                          int win_h, int P1, int P2, uint8_t *ws, uint8_t *disp, hipStream_t s)
{
    sv_status r = launch_zncc_cost(ll, lr, B, h, w, D, sgm_dpad(D), win_w, win_h, ws, s);
    if (r != SV_OK) return r;
    return sgm_from_cost(B, h, w, D, P1, P2, ws, disp, s);
}

sv_status launch_smp_median(const uint8_t *disp, int B, int h, int w, int D, uint8_t *tmp,
                            uint8_t *out, hipStream_t s)
{
    if (w > SMP_MAXW) return SV_ERR_SHAPE;
    hipLaunchKernelGGL(k_smp, dim3(B * h), dim3(64), 0, s, disp, B, h, w, D, tmp);
    SV_LAUNCH_CHECK("k_smp");
    const size_t n = (size_t)B * h * w;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_median3, dim3(blocks), dim3(256), 0, s, tmp, B, h, w, out);
    SV_LAUNCH_CHECK("k_median3");
    return SV_OK;
}

}  // namespace sv
