// Training-side kernels: the loss (a reading of Eqs. (9)-(11)) with its
// gradient, and the Adam update of Sec. IV-A.  Reductions use a fixed grid
// and a fixed tree order (FP64 partial sums), so results do not depend on
// scheduling.
#include "kernels.h"

namespace sv {

constexpr int LOSS_BLOCKS = 512, LOSS_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = LOSS_THREADS / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Each block owns a contiguous slice of the pixels and of the latent elements.
__global__ void __launch_bounds__(LOSS_THREADS)
k_loss_partial(const float *__restrict__ out, const float *__restrict__ gt, int64_t n,
               const float *__restrict__ ml, int64_t npix_lat, int L, float *__restrict__ dout,
               double *__restrict__ part)
{
    __shared__ double sh[LOSS_THREADS];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    const float inv_n = 1.0f / (float)n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += LOSS_THREADS) {
        const float e = out[i] - gt[i];
        const float a = fabsf(e);
        s += a < 1.0f ? 0.5 * (double)e * e : (double)a - 0.5;
        if (dout) dout[i] = fminf(fmaxf(e, -1.0f), 1.0f) * inv_n;
    }
    const double data = block_sum(s, sh);
    const int64_t nl = npix_lat * L;
    const int64_t perl = (nl + gridDim.x - 1) / gridDim.x;
    const int64_t llo = blockIdx.x * perl, lhi = llo + perl < nl ? llo + perl : nl;
    double k = 0.0;
    for (int64_t i = llo + threadIdx.x; i < lhi; i += LOSS_THREADS) {
        const int64_t p = i / L;
        const int c = (int)(i - p * L);
        const double mu = ml[p * 2 * L + c], lv = ml[p * 2 * L + L + c];
        k += 0.5 * (mu * mu + exp(lv) - 1.0 - lv);
    }
    const double kl = block_sum(k, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = data;
        part[2 * blockIdx.x + 1] = kl;
    }
}

__global__ void __launch_bounds__(LOSS_THREADS)
k_loss_final(const double *__restrict__ part, int nblocks, int64_t n, int64_t nl, float klw,
             float *__restrict__ loss_out)
{
    __shared__ double sh[LOSS_THREADS];
    double d = 0.0, k = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += LOSS_THREADS) {
        d += part[2 * i];
        k += part[2 * i + 1];
    }
    d = block_sum(d, sh);
    k = block_sum(k, sh);
    if (threadIdx.x == 0) {
        const double data = d / (double)n, kl = nl > 0 ? k / (double)nl : 0.0;
        loss_out[0] = (float)(data + klw * kl);
        loss_out[1] = (float)data;
        loss_out[2] = (float)kl;
    }
}

size_t loss_workspace_bytes() { return sizeof(double) * 2 * LOSS_BLOCKS; }

sv_status launch_loss(const float *out, const float *gt, int64_t n, const float *ml,
                      int64_t npix_lat, int L, float klw, float *loss_out, float *dout, void *ws,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_loss_partial, dim3(LOSS_BLOCKS), dim3(LOSS_THREADS), 0, s, out, gt, n, ml,
                       ml ? npix_lat : 0, L, dout, (double *)ws);
    SV_LAUNCH_CHECK("k_loss_partial");
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(LOSS_THREADS), 0, s, (const double *)ws,
                       LOSS_BLOCKS, n, ml ? npix_lat * L : 0, klw, loss_out);
    SV_LAUNCH_CHECK("k_loss_final");
    return SV_OK;
}

// Adam with bias correction; FP32 master weights and moments.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

sv_status launch_adam(float *w, const float *g, float *m, float *v, int64_t n, int step, float lr,
                      float b1, float b2, float eps, hipStream_t s)
{
    const float bc1 = (float)(1.0 - pow((double)b1, step));
    const float bc2 = (float)(1.0 - pow((double)b2, step));
    const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2,
                       eps, bc1, bc2);
    SV_LAUNCH_CHECK("k_adam");
    return SV_OK;
}

}  // namespace sv

using namespace sv;

extern "C" {

size_t sv_loss_workspace_bytes(void) { return loss_workspace_bytes(); }

sv_status sv_loss(const float *out, const float *gt, int64_t n, const float *mu_logvar,
                  int64_t n_pix_lat, int latent, float kl_weight, float *loss_out, float *dout,
                  void *workspace, size_t ws_bytes, void *stream)
{
    if (!out || !gt || !loss_out || !workspace) return SV_ERR_NULL;
    if (n <= 0 || n_pix_lat < 0 || (mu_logvar && latent <= 0)) return SV_ERR_SHAPE;
    if (ws_bytes < loss_workspace_bytes()) return SV_ERR_WORKSPACE;
    if ((uintptr_t)workspace % 8) return SV_ERR_RANGE;
    return launch_loss(out, gt, n, mu_logvar, n_pix_lat, latent, kl_weight, loss_out, dout,
                       workspace, (hipStream_t)stream);
}

sv_status sv_adam_step(float *w, const float *g, float *m, float *v, int64_t n, int step,
                       float lr, float beta1, float beta2, float eps, void *stream)
{
    if (!w || !g || !m || !v) return SV_ERR_NULL;
    if (n <= 0) return SV_ERR_SHAPE;
    if (step < 1 || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return SV_ERR_RANGE;
    return launch_adam(w, g, m, v, n, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}

}  // extern "C"
