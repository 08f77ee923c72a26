// Latent head and first decoder layer of an inference pass in one kernel.
//
// At inference the latent code is the mean (Eq. (8) without the noise term):
// [mu | logvar] = 1x1 convolution of E3, then G3 = leaky ReLU of a 1x1
// convolution of mu.  Both layers are pointwise in the pixels, so one
// workgroup owns 16 pixels of the coarsest level for both: E3's channels, and
// then mu, sit in LDS, and each wave takes 16-channel output blocks (with few
// pixels, two workgroups share the 16: one computes mu and G3, the other
// logvar, halving the longest chain of blocks a wave runs).  The
// reduction runs over the input channels in base chunks in ascending order
// with the same MFMA steps as the unsplit convolution kernel, and the values
// go through the same epilogue and the same conversion into the compute dtype,
// so the result has the same bits as the two layers launched one by one.
#include "conv_impl.h"

namespace sv {

constexpr int LAT_THREADS = 512;
constexpr int LAT_PX = 16;     // pixels per workgroup (one MFMA block)
constexpr int LAT_MAXC = 256;  // most channels of E3 and of mu held in LDS

template <int DT>
__global__ void __launch_bounds__(LAT_THREADS) k_latent(const ConvParams ph, const ConvParams pg, int npix,
                                                        const float *__restrict__ e3part, int e3split,
                                                        const float *__restrict__ e3bias, int roles)
{
    using M = Mfma<DT>;
    using T = typename M::T;
    using vec = typename M::vec;
    constexpr int GS = M::GS;
    constexpr int KCB = DT == SV_F32 ? 16 : 32;
    constexpr int KP = LAT_MAXC + GS;  // LDS row in elements (16-byte multiple)
    constexpr int NWAVE = LAT_THREADS / 64;
    __shared__ __attribute__((aligned(16))) T xs[LAT_PX * KP];  // E3 of the pixels
    __shared__ __attribute__((aligned(16))) T zs[LAT_PX * KP];  // mu of the pixels
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    // few pixels (small batches): two workgroups per 16 pixels, role 0
    // computing mu and then G3, role 1 logvar, so that each wave's chain
    // holds at most two output blocks; else one workgroup does all (role -1)
    const int role = roles == 2 ? (int)(blockIdx.x & 1) : -1;
    const int p0 = (roles == 2 ? blockIdx.x >> 1 : blockIdx.x) * LAT_PX, pix = p0 + r16;
    const int c3 = ph.Cin, L = pg.Cin;

    // E3 -> LDS; pixels past npix are zero and their results are not stored.
    // From a deferred split: the ranges' partials added in range order, then
    // bias and leaky ReLU, rounded to the compute dtype -- the second pass of
    // the split and E3's store, as the convolution kernels do them.
    {
        const T *e3 = (const T *)ph.src[0].ptr;
        const int ngrp = c3 / GS;
        for (int e = tid; e < LAT_PX * ngrp; e += LAT_THREADS) {
            const int r = e / ngrp, cg = e - r * ngrp;
            vec v;
            if (p0 + r < npix && e3split > 1) {
                const size_t o = (size_t)(p0 + r) * c3 + cg * GS;
                float a[GS];
#pragma unroll
                for (int i = 0; i < GS; i += 4) {
                    f32x4 q[CONV_MAX_SPLIT];
#pragma unroll
                    for (int z = 0; z < CONV_MAX_SPLIT; ++z) {
                        const size_t zz = z < e3split ? (size_t)z : 0;
                        q[z] = *(const f32x4 *)&e3part[zz * npix * c3 + o + i];
                    }
                    f32x4 s = q[0];
#pragma unroll
                    for (int z = 1; z < CONV_MAX_SPLIT; ++z) {
                        if (z < e3split) {
                            s[0] += q[z][0]; s[1] += q[z][1]; s[2] += q[z][2]; s[3] += q[z][3];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        float val = s[j] + e3bias[cg * GS + i + j];
                        val = val > 0.f ? val : 0.1f * val;
                        a[i + j] = val;
                    }
                }
#pragma unroll
                for (int i = 0; i < GS; ++i) v[i] = Elem<DT>::make(a[i]);
            } else if (p0 + r < npix) {
                v = *(const vec *)(e3 + (size_t)(p0 + r) * ph.src[0].pitch + cg * GS);
            } else {
#pragma unroll
                for (int i = 0; i < GS; ++i) v[i] = 0;
            }
            *(vec *)&xs[r * KP + cg * GS] = v;
        }
    }
    __syncthreads();

    // head: output block blk of 16 channels of [mu | logvar]
    {
        const T *w = (const T *)ph.wpk;
        const int nblk = ph.n_pad / 16, nkb = c3 / KCB, nmu = L / 16;
        for (int blk = wave + (role == 1 ? nmu : 0); blk < (role == 0 ? nmu : nblk); blk += NWAVE) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const T *wr = w + (size_t)(blk * 16 + r16) * ph.cin_pad + g * GS;
            const T *xr = xs + r16 * KP + g * GS;
#pragma unroll 4
            for (int kb = 0; kb < nkb; ++kb)
                acc = M::run(*(const vec *)(wr + kb * KCB), *(const vec *)(xr + kb * KCB), acc);
            const int nbase = blk * 16 + 4 * g;
            float bias[4];
            conv_bias4<DT>(ph, nbase, bias);
            const float r[4] = {acc[0], acc[1], acc[2], acc[3]};
            if (pix < npix) conv_epilogue<DT>(ph, (size_t)pix, nbase, r, bias);
            // mu in the compute dtype, as the G3 layer stages it from the FP32 map
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (nbase + i < L) zs[r16 * KP + nbase + i] = Elem<DT>::make(r[i] + bias[i]);
        }
    }
    if (role == 1) return;
    __syncthreads();

    // G3: output block blk of 16 channels
    {
        const T *w = (const T *)pg.wpk;
        const int nblk = pg.n_pad / 16, nkb = L / KCB;
        for (int blk = wave; blk < nblk; blk += NWAVE) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const T *wr = w + (size_t)(blk * 16 + r16) * pg.cin_pad + g * GS;
            const T *zr = zs + r16 * KP + g * GS;
#pragma unroll 4
            for (int kb = 0; kb < nkb; ++kb)
                acc = M::run(*(const vec *)(wr + kb * KCB), *(const vec *)(zr + kb * KCB), acc);
            const int nbase = blk * 16 + 4 * g;
            float bias[4];
            conv_bias4<DT>(pg, nbase, bias);
            const float r[4] = {acc[0], acc[1], acc[2], acc[3]};
            if (pix < npix) conv_epilogue<DT>(pg, (size_t)pix, nbase, r, bias);
        }
    }
}

bool latent_fusable(int dtype, int c3, int L) {
    if (dtype != SV_F32 && dtype != SV_BF16 && dtype != SV_F16) return false;
    const int kcb = dtype == SV_F32 ? 16 : 32;
    return c3 > 0 && L > 0 && c3 % kcb == 0 && L % kcb == 0 && c3 <= LAT_MAXC && L <= LAT_MAXC;
}

sv_status launch_latent(int dtype, const ConvParams &ph, const ConvParams &pg, int npix,
                        const float *e3part, int e3split, const float *e3bias, hipStream_t st) {
    const int c3 = ph.Cin, L = pg.Cin;
    // shapes the kernel assumes: both reductions whole base chunks held in
    // LDS, mu the first L of the head's outputs, G3 reading exactly mu, and
    // packed rows long enough for every chunk
    if (!latent_fusable(dtype, c3, L) || ph.Cout != 2 * L || pg.Cout != c3 ||
        ph.cin_pad < c3 || pg.cin_pad < L || ph.n_pad < ph.Cout || pg.n_pad < pg.Cout ||
        ph.n_pad % 16 || pg.n_pad % 16 || ph.src[0].pitch < c3 || !ph.out_f32 ||
        e3split > CONV_MAX_SPLIT || (e3split > 1 && (!e3part || !e3bias)))
        return SV_ERR_UNSUPPORTED;
    if (npix <= 0) return SV_OK;
    const int groups = cdiv(npix, LAT_PX);
    const int roles = groups < 256 ? 2 : 1;  // two roles while the groups leave CUs idle
    const dim3 grid((unsigned)(roles * groups));
    switch (dtype) {
    case SV_F32: hipLaunchKernelGGL(k_latent<SV_F32>, grid, dim3(LAT_THREADS), 0, st, ph, pg, npix, e3part, e3split, e3bias, roles); break;
    case SV_BF16: hipLaunchKernelGGL(k_latent<SV_BF16>, grid, dim3(LAT_THREADS), 0, st, ph, pg, npix, e3part, e3split, e3bias, roles); break;
    default: hipLaunchKernelGGL(k_latent<SV_F16>, grid, dim3(LAT_THREADS), 0, st, ph, pg, npix, e3part, e3split, e3bias, roles); break;
    }
    SV_LAUNCH_CHECK("k_latent");
    return SV_OK;
}

}  // namespace sv
