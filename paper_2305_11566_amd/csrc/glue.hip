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
__device__ __forceinline__ void final_px(const float *__restrict__ Tb, int tpitch,
                                         const uint8_t *__restrict__ db, float scale0, float bias,
                                         int h, int w, int H, int W, int X, int Y,
                                         float *__restrict__ out)
{
    float acc = bias;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const int yy = Y + u - 1;
        if (yy < 0 || yy >= H) continue;
        int y0, y1;
        float ly;
        bilin(yy, h, H, y0, y1, ly);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const int xx = X + v - 1;
            if (xx < 0 || xx >= W) continue;
            int x0, x1;
            float lx;
            bilin(xx, w, W, x0, x1, lx);
            const int t = u * 3 + v;
            const float a00 = Tb[((size_t)y0 * w + x0) * tpitch + t];
            const float a01 = Tb[((size_t)y0 * w + x1) * tpitch + t];
            const float a10 = Tb[((size_t)y1 * w + x0) * tpitch + t];
            const float a11 = Tb[((size_t)y1 * w + x1) * tpitch + t];
            const float top = (1.f - lx) * a00 + lx * a01;
            const float bot = (1.f - lx) * a10 + lx * a11;
            acc += (1.f - ly) * top + ly * bot;
        }
    }
    int y0, y1, x0, x1;
    float ly, lx;
    bilin(Y, h, H, y0, y1, ly);
    bilin(X, w, W, x0, x1, lx);
    const float top = (1.f - lx) * (float)db[(size_t)y0 * w + x0] + lx * (float)db[(size_t)y0 * w + x1];
    const float bot = (1.f - lx) * (float)db[(size_t)y1 * w + x0] + lx * (float)db[(size_t)y1 * w + x1];
    const float base = scale0 * ((1.f - ly) * top + ly * bot);
    out[(size_t)Y * W + X] = 256.0f * (acc + base);
}

__global__ void __launch_bounds__(256)
k_final(const float *__restrict__ T, int tpitch, const uint8_t *__restrict__ disp, float scale0,
        const float *__restrict__ biasF, int h, int w, int H, int W, float *__restrict__ out)
{
    const int X = blockIdx.x * FIN_TILE_W + (threadIdx.x & 63);
    const int Y = blockIdx.y * FIN_TILE_H + (threadIdx.x >> 6);
    const int b = blockIdx.z;
    if (X >= W || Y >= H) return;
    final_px(T + (size_t)b * h * w * tpitch, tpitch, disp + (size_t)b * h * w, scale0, biasF[0], h,
             w, H, W, X, Y, out + (size_t)b * H * W);
}

// Persistent variant over the pair table; each pair writes its own output map.
__global__ void __launch_bounds__(256)
k_final_tab(const PairTable *__restrict__ tab, const float *__restrict__ T, int tpitch,
            const uint8_t *__restrict__ disp, float scale0, const float *__restrict__ biasF)
{
    const int n = tab->n;
    const int *cum = tab->cum[BS_FINAL];
    const int total = cum[n];
    const float bias = biasF[0];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = table_find(cum, n, t);
        const PairGeo &g = tab->pair[i];
        const int local = t - cum[i];
        const int tx = cdiv_d(g.W, FIN_TILE_W);
        const int X = (local % tx) * FIN_TILE_W + (threadIdx.x & 63);
        const int Y = (local / tx) * FIN_TILE_H + (threadIdx.x >> 6);
        if (X < g.W && Y < g.H)
            final_px(T + (size_t)g.off[0] * tpitch, tpitch, disp + g.off[0], scale0, bias, g.h[0],
                     g.w[0], g.H, g.W, X, Y, g.out);
    }
}

sv_status launch_final_tab(const PairTable *tab, int grid, const float *T, int tpitch,
                           const uint8_t *disp, float scale0, const float *biasF, hipStream_t s)
{
    hipLaunchKernelGGL(k_final_tab, dim3(grid), dim3(256), 0, s, tab, T, tpitch, disp, scale0, biasF);
    SV_LAUNCH_CHECK("k_final_tab");
    return SV_OK;
}

sv_status launch_final(const float *T, int tpitch, const uint8_t *disp, float scale0,
                       const float *biasF, int B, int h, int w, int H, int W, float *out,
                       hipStream_t s)
{
    dim3 grid(cdiv(W, FIN_TILE_W), cdiv(H, FIN_TILE_H), B);
    hipLaunchKernelGGL(k_final, grid, dim3(256), 0, s, T, tpitch, disp, scale0, biasF, h, w, H, W,
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
