// Network glue: the final upsampling layer and the reparameterisation.
#include "kernels.h"

namespace sv {

// Final layer (Table I, "UP-SAMPLING"): R = conv3x3(resize([G0, x0] -> H x W))
// to one channel, plus the bilinear upscaling of the coarse map (the paper's
// "Mini+Linear" baseline, Sec. IV-C) as the residual base.  Convolution and
// resize are both linear, so with T_t(i) = sum_c W[c, t] X[c](i) computed at
// the coarse level (one 1x1 output channel per tap t = (u, v)),
//   R(Y, X) = sum_t [inside] resize(T_t)(Y + u - 1, X + v - 1).
// Each full-resolution pixel then gathers 9 bilinear samples of the 9-channel
// map T instead of 3 x 3 x (c1 + 2) upsampled values.
//
// One workgroup = FIN_TILE_W x FIN_TILE_H output pixels.  The bilinear indices
// and weights of the tile's FIN_TILE_W + 2 columns and FIN_TILE_H + 2 rows
// (the 3 x 3 neighbourhood reaches one pixel past each edge) are computed once
// into LDS, together with the coarse window of T and of the coarse disparity
// that the tile touches; every pixel then reads only LDS.  Since w <= W, the
// lower bilinear index grows by at most one per output pixel, which bounds
// the coarse window by (FIN_TILE_W + 3) x (FIN_TILE_H + 3).
constexpr int FIN_CX = FIN_TILE_W + 2, FIN_CY = FIN_TILE_H + 2;
constexpr int FIN_PW = FIN_TILE_W + 3, FIN_PH = FIN_TILE_H + 3;
constexpr int FIN_THREADS = 256;
static_assert(FIN_TILE_W == 64 && FIN_TILE_H % (FIN_THREADS / 64) == 0, "final tile shape");

struct FinSmem {
    float T[9][FIN_PH][FIN_PW];
    float d[FIN_PH][FIN_PW];
    int cx0[FIN_CX], cx1[FIN_CX], cy0[FIN_CY], cy1[FIN_CY];  // -1: outside the image
    float clx[FIN_CX], cly[FIN_CY];
};

__device__ __forceinline__ void final_tile(FinSmem &sm, const float *__restrict__ Tb, int tpitch,
                                           const uint8_t *__restrict__ db, float scale0,
                                           float bias, int h, int w, int H, int W, int X0,
                                           int Y0, float *__restrict__ out)
{
    const int tid = threadIdx.x;
    // coarse window origin: the lower index of the first column / row in range
    int xa, ya, i1;
    float lam;
    bilin(max(X0 - 1, 0), w, W, xa, i1, lam);
    bilin(max(Y0 - 1, 0), h, H, ya, i1, lam);
    int xb, yb;
    bilin(min(X0 + FIN_TILE_W, W - 1), w, W, i1, xb, lam);
    bilin(min(Y0 + FIN_TILE_H, H - 1), h, H, i1, yb, lam);
    const int pw = xb - xa + 1, ph = yb - ya + 1;
    if (tid < FIN_CX) {
        const int X = X0 - 1 + tid;
        int x0 = -1, x1 = -1;
        float lx = 0.f;
        if (X >= 0 && X < W) {
            bilin(X, w, W, x0, x1, lx);
            x0 -= xa;
            x1 -= xa;
        }
        sm.cx0[tid] = x0;
        sm.cx1[tid] = x1;
        sm.clx[tid] = lx;
    } else if (tid >= 128 && tid < 128 + FIN_CY) {
        const int r = tid - 128, Y = Y0 - 1 + r;
        int y0 = -1, y1 = -1;
        float ly = 0.f;
        if (Y >= 0 && Y < H) {
            bilin(Y, h, H, y0, y1, ly);
            y0 -= ya;
            y1 -= ya;
        }
        sm.cy0[r] = y0;
        sm.cy1[r] = y1;
        sm.cly[r] = ly;
    }
    for (int e = tid; e < ph * pw * 9; e += FIN_THREADS) {
        const int t = e % 9, q = e / 9;
        const int r = q / pw, c = q - r * pw;
        sm.T[t][r][c] = Tb[((size_t)(ya + r) * w + xa + c) * tpitch + t];
    }
    for (int e = tid; e < ph * pw; e += FIN_THREADS) {
        const int r = e / pw, c = e - r * pw;
        sm.d[r][c] = (float)db[(size_t)(ya + r) * w + xa + c];
    }
    __syncthreads();
    const int tx = tid & 63;
    const int X = X0 + tx;
#pragma unroll
    for (int ty = tid >> 6; ty < FIN_TILE_H; ty += FIN_THREADS / 64) {
        const int Y = Y0 + ty;
        if (X < W && Y < H) {
            float acc = bias;
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int y0 = sm.cy0[ty + u];
                if (y0 < 0) continue;
                const int y1 = sm.cy1[ty + u];
                const float ly = sm.cly[ty + u];
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    const int x0 = sm.cx0[tx + v];
                    if (x0 < 0) continue;
                    const int x1 = sm.cx1[tx + v];
                    const float lx = sm.clx[tx + v];
                    const int t = u * 3 + v;
                    const float top = (1.f - lx) * sm.T[t][y0][x0] + lx * sm.T[t][y0][x1];
                    const float bot = (1.f - lx) * sm.T[t][y1][x0] + lx * sm.T[t][y1][x1];
                    acc += (1.f - ly) * top + ly * bot;
                }
            }
            const int y0 = sm.cy0[ty + 1], y1 = sm.cy1[ty + 1];
            const int x0 = sm.cx0[tx + 1], x1 = sm.cx1[tx + 1];
            const float ly = sm.cly[ty + 1], lx = sm.clx[tx + 1];
            const float top = (1.f - lx) * sm.d[y0][x0] + lx * sm.d[y0][x1];
            const float bot = (1.f - lx) * sm.d[y1][x0] + lx * sm.d[y1][x1];
            const float base = scale0 * ((1.f - ly) * top + ly * bot);
            out[(size_t)Y * W + X] = 256.0f * (acc + base);
        }
    }
    __syncthreads();  // the LDS is reused by the next tile of a persistent loop
}

__global__ void __launch_bounds__(FIN_THREADS)
k_final(const float *__restrict__ T, int tpitch, const uint8_t *__restrict__ disp, float scale0,
        const float *__restrict__ biasF, int h, int w, int H, int W, float *__restrict__ out)
{
    __shared__ FinSmem sm;
    const int b = blockIdx.z;
    final_tile(sm, T + (size_t)b * h * w * tpitch, tpitch, disp + (size_t)b * h * w, scale0,
               biasF[0], h, w, H, W, blockIdx.x * FIN_TILE_W, blockIdx.y * FIN_TILE_H,
               out + (size_t)b * H * W);
}

// Persistent variant over the pair table; each pair writes its own output map.
__global__ void __launch_bounds__(FIN_THREADS)
k_final_tab(const PairTable *__restrict__ tab, const float *__restrict__ T, int tpitch,
            const uint8_t *__restrict__ disp, float scale0, const float *__restrict__ biasF)
{
    __shared__ FinSmem sm;
    const int n = tab->n;
    const int *cum = tab->cum[BS_FINAL];
    const int total = cum[n];
    const float bias = biasF[0];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = table_find(cum, n, t);
        const PairGeo &g = tab->pair[i];
        const int local = t - cum[i];
        const int tx = cdiv_d(g.W, FIN_TILE_W);
        final_tile(sm, T + (size_t)g.off[0] * tpitch, tpitch, disp + g.off[0], scale0, bias,
                   g.h[0], g.w[0], g.H, g.W, (local % tx) * FIN_TILE_W, (local / tx) * FIN_TILE_H,
                   g.out);
    }
}

sv_status launch_final_tab(const PairTable *tab, int grid, const float *T, int tpitch,
                           const uint8_t *disp, float scale0, const float *biasF, hipStream_t s)
{
    hipLaunchKernelGGL(k_final_tab, dim3(grid), dim3(FIN_THREADS), 0, s, tab, T, tpitch, disp, scale0, biasF);
    SV_LAUNCH_CHECK("k_final_tab");
    return SV_OK;
}

sv_status launch_final(const float *T, int tpitch, const uint8_t *disp, float scale0,
                       const float *biasF, int B, int h, int w, int H, int W, float *out,
                       hipStream_t s)
{
    dim3 grid(cdiv(W, FIN_TILE_W), cdiv(H, FIN_TILE_H), B);
    hipLaunchKernelGGL(k_final, grid, dim3(FIN_THREADS), 0, s, T, tpitch, disp, scale0, biasF, h, w, H, W,
                       out);
    SV_LAUNCH_CHECK("k_final");
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
