/*
 * sv.h -- C ABI of libsv.so, the MI355X (gfx950) hot path of StereoVAE
 * (Chang et al., "StereoVAE: A lightweight stereo-matching system using
 * embedded GPUs", arXiv 2305.11566).
 *
 * A rectified uint8 stereo pair goes in, a dense full-resolution disparity
 * map comes out (the problem statement of Sec. I and Sec. III-B1): the pair is
 * reduced by a factor f, matched by census + Hamming cost + winner-take-all
 * at the reduced resolution, and the tiny VAE of Table I upsamples and refines
 * the coarse map.
 *
 * Conventions shared by every entry point
 *  - Pointers marked (device) are device memory owned by the caller; pointers
 *    marked (host) are read during the call only.  The library never
 *    allocates inside these calls, except sv_batch_plan_create/_destroy and
 *    sv_autotune, which own what they allocate.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every
 *    call is asynchronous on it and returns without waiting for the device,
 *    except the calls that say otherwise: sv_autotune and sv_tvae_autotune
 *    (they time kernels), sv_profile_read (it reads the recorded events),
 *    sv_batch_plan_destroy, and sv_stereo_batch only when the plan's ring of
 *    pinned pair tables wraps onto a table whose upload is still in flight.
 *  - Calls are re-entrant: several threads may call any entry point at once
 *    on their own buffers and streams.  The process-wide settings
 *    (sv_set_layer_cfg, sv_set_cost_wta_split, sv_set_latent_fusion,
 *    sv_tvae_set_layer_cfg, sv_tvae_set_deconv_form, sv_profile_enable) are
 *    atomic and apply to calls that start after the setter returns; the
 *    autotuners pass the configurations they time with each call and change
 *    no such setting; the autotune caches are guarded by a mutex.  A batch
 *    plan is one mutable object: one thread at a time per plan.
 *  - All arguments are validated before anything is enqueued, and validation
 *    makes no HIP call; a failed check returns a negative code and enqueues
 *    nothing.  A HIP launch error is returned as SV_ERR_HIP; errors raised
 *    later on the device surface on a later call or at synchronisation.
 *  - Image layouts are row-major; network tensors are NHWC.  Disparities are
 *    in pixels of the resolution they are stored at, the left view is the
 *    reference and a left pixel x matches right pixel x - d.
 *  - Integer results are bitwise deterministic; floating-point results are
 *    deterministic for a fixed tile configuration (no floating-point atomics).
 */
#ifndef SV_H_
#define SV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sv_status;

#define SV_OK 0
#define SV_ERR_NULL (-1)        /* a required pointer is NULL */
#define SV_ERR_SHAPE (-2)       /* a size is non-positive or inconsistent */
#define SV_ERR_RANGE (-3)       /* a parameter is outside its supported range */
#define SV_ERR_DTYPE (-4)       /* unknown dtype code */
#define SV_ERR_WORKSPACE (-5)   /* workspace / saved buffer smaller than required */
#define SV_ERR_UNSUPPORTED (-6) /* valid but not supported by this build */
#define SV_ERR_HIP (-7)         /* the HIP runtime reported an error */

/* Compute / storage precision of the network's convolutions.  Accumulation is
 * FP32 for SV_F32 / SV_BF16 / SV_F16; the residual base, the latent, KL and
 * loss stay FP32.
 * SV_I8 (the configurable network's sv_vae_* inference only): the quantised
 * network that the paper's closing section plans -- INT8 weights with one
 * scale per output channel (code = clamp(rint(w * 127 / a), -127, 127), a =
 * max |w| of the channel) and INT8 activations with one dynamic scale per
 * tensor (every convolution's epilogue records max |stored value| of its
 * output; a layer quantises what it reads with 127 / m, m the largest amax of
 * its sources; x0's amax comes from the coarse maps), exact INT32 sums on the
 * MFMA units (E1, two input channels: the same exact sums in a direct
 * stencil), then y = float(sum) * (s_in * s_w) + bias in FP32, activations
 * stored in BF16.  The final layer keeps FP32 weights as in every mode (at
 * inference applied by G0's epilogue to the BF16-rounded G0, as for the
 * 16-bit types). */
#define SV_F32 0
#define SV_BF16 1
#define SV_F16 2
#define SV_I8 3

/* Human-readable name of a status code (static storage). */
const char *sv_status_str(sv_status s);

/* Last HIP error text seen by this thread (static per thread). */
const char *sv_last_error(void);

/* ------------------------------------------------------------------------ */
/* Coarse matching (Sec. III-A)                                              */
/* ------------------------------------------------------------------------ */

/*
 * Reduce and census-transform a batch of images.
 *
 * Reduction ("small image pairs", Sec. IV-C; quarter-size inputs, Table I):
 * low[b][i][j] = round-half-up mean of the in-bounds pixels of the f x f block
 * at (f*i, f*j), for i < h = ceil(H/f), j < w = ceil(W/f); f = 1 copies.
 * Census (named in Sec. I and Sec. III; variants S1/S2 of Sec. IV-C): for a
 * win_w x win_h window (both odd), neighbours enumerated row by row skipping
 * the centre, bit k of census[b][i][j] is 1 when neighbour k is strictly
 * smaller than the centre; borders clamp to the edge; nbits = win_w*win_h - 1
 * <= 64 and higher bits are 0.
 *
 * img        (device) uint8 [B][H][pitch], pitch >= W bytes per row
 * factor     1..8
 * low_out    (device, nullable) uint8 [B][h][w]
 * census_out (device) uint64 [B][h][w]
 * Errors: SV_ERR_NULL (img, census_out), SV_ERR_SHAPE (B,H,W <= 0, pitch < W),
 *         SV_ERR_RANGE (factor, even or < 1 window, nbits > 64).
 */
sv_status sv_census(const uint8_t *img, int B, int H, int W, int pitch, int factor, int win_w,
                    int win_h, uint8_t *low_out, uint64_t *census_out, void *stream);

/*
 * Both views of a batch of pairs in one launch: same contract as sv_census
 * applied to `left` (reduced image written to low_left when non-NULL) and to
 * `right`.
 */
sv_status sv_census_pair(const uint8_t *left, const uint8_t *right, int B, int H, int W,
                         int pitch, int factor, int win_w, int win_h, uint8_t *low_left,
                         uint64_t *cen_left, uint64_t *cen_right, void *stream);

/*
 * Hamming matching cost and winner-take-all, Eq. (6).
 *
 * cost(i, j, d) = popcount(cen_l[i][j] XOR cen_r[i][j-d]) for j-d >= 0, and
 * nbits + 1 when j - d < 0 (the target column of Eq. (1) leaves the image);
 * disp_out[b][i][j] = the least-cost d in [0, D), the lowest d on ties.  The
 * cost volume is never stored.
 *
 * cen_l, cen_r (device) uint64 [B][h][w]
 * D            1..256;  nbits 1..64
 * disp_out     (device) uint8 [B][h][w], in reduced-resolution pixels
 * Errors: SV_ERR_NULL, SV_ERR_SHAPE, SV_ERR_RANGE (D, nbits).
 */
sv_status sv_cost_wta(const uint64_t *cen_l, const uint64_t *cen_r, int B, int h, int w, int D,
                      int nbits, uint8_t *disp_out, void *stream);

/* Lanes per pixel of the cost + WTA kernel for all later calls: 1, 2, 4 or 8
 * (lane k of a pixel sweeps d = k, k + split, ...), or 0 (the default) for
 * the per-shape choice -- the split sv_autotune timed fastest for this
 * (B, h, w, D) in this process, else 4.  The result does not depend on it.
 * Process-wide, atomic.  Errors: SV_ERR_RANGE. */
sv_status sv_set_cost_wta_split(int dsplit);

/* ------------------------------------------------------------------------ */
/* Semi-global matching and post-processing (Sec. III-A2, III-A3)             */
/* ------------------------------------------------------------------------ */

/* Bytes of workspace sv_sgm needs: the matching-cost volume and the four
 * path-cost volumes, uint8 each, 5 * B*h*w*Dp with Dp = D rounded up to a
 * multiple of 4. */
size_t sv_sgm_workspace_bytes(int B, int h, int w, int D);

/*
 * Semi-global matching on the census cost, Eqs. (4)-(6): with C(i, j, d) the
 * cost of sv_cost_wta, the path cost along direction r is
 *   C_r(p, d) = C(p, d) + min(C_r(p-r, d), C_r(p-r, d-1) + P1,
 *                             C_r(p-r, d+1) + P1, min_i C_r(p-r, i) + P2)
 *               - min_k C_r(p-r, k),
 * starting from C_r = C at the first pixel of each path, over the four axis
 * directions (left to right, right to left, top to bottom, bottom to top);
 * disp_out is the argmin over d of the sum of the four (Eq. (5)), the lowest
 * d on ties.  Integer arithmetic throughout: bit-exact.
 *
 * cen_l, cen_r (device) uint64 [B][h][w]; D 1..256; nbits 1..64
 * P1, P2       penalties, 0 <= P1 <= P2 and nbits + 1 + P2 <= 255 (path costs
 *              are kept as uint8)
 * disp_out     (device) uint8 [B][h][w]
 * workspace    (device) >= sv_sgm_workspace_bytes(B, h, w, D) bytes, caller-owned
 * Errors: SV_ERR_NULL, SV_ERR_SHAPE, SV_ERR_RANGE (D, nbits, P1, P2),
 *         SV_ERR_WORKSPACE.
 */
sv_status sv_sgm(const uint64_t *cen_l, const uint64_t *cen_r, int B, int h, int w, int D,
                 int nbits, int P1, int P2, uint8_t *disp_out, void *workspace, size_t ws_bytes,
                 void *stream);

/*
 * Zero-mean normalised cross-correlation + SGM (Eqs. (1)-(6)): the paper's
 * main coarse matcher, on the reduced images.  With the window clamped to the
 * image edge and n = win_w * win_h,
 *   C(i, j, d) = 1 - N / sqrt(A B),  N = n SRT - SR ST,  A = n SRR - SR^2,
 *                B = n STT - ST^2
 * over the window sums of reference (R = low_l around (i, j)) and target
 * (T = low_r around (i, j - d)) values, C = 1 for a flat window and C = 2 when
 * j - d < 0; the integer cost q = floor(32 C + 1/2) (0..64, FP64) feeds the
 * path aggregation of sv_sgm with penalties P1, P2 in the same units, and
 * disp_out is the WTA of the aggregated cost.  Bit-exact.
 *
 * low_l, low_r (device) uint8 [B][h][w] reduced images (e.g. sv_census's low_out)
 * D 1..256; windows 3x3, 5x5, 7x7, 9x7 (9 wide), 7x9, 9x9, 5x3, 3x5
 * P1, P2       0 <= P1 <= P2 <= 190
 * disp_out     (device) uint8 [B][h][w]
 * workspace    >= sv_sgm_workspace_bytes(B, h, w, D)
 * Errors: SV_ERR_NULL, SV_ERR_SHAPE, SV_ERR_RANGE, SV_ERR_UNSUPPORTED (window),
 *         SV_ERR_WORKSPACE.
 */
sv_status sv_zncc_sgm(const uint8_t *low_l, const uint8_t *low_r, int B, int h, int w, int D,
                      int win_w, int win_h, int P1, int P2, uint8_t *disp_out, void *workspace,
                      size_t ws_bytes, void *stream);

/* The integer ZNCC cost q of sv_zncc_sgm alone, uint8 [B][h][w][D] (device,
 * caller-owned cost_out).  Same arguments and errors. */
sv_status sv_zncc_cost(const uint8_t *low_l, const uint8_t *low_r, int B, int h, int w, int D,
                       int win_w, int win_h, uint8_t *cost_out, void *stream);

/* Bytes of workspace sv_smp_median needs: B*h*w. */
size_t sv_smp_workspace_bytes(int B, int h, int w);

/*
 * Single matching phase (Eq. (7)) and a 3 x 3 median filter.  The target
 * column of pixel (i, j) is j - disp_in[i][j]; no target column may be matched
 * twice, and of two pixels j < j' of a row with the same target column the
 * left one (the smaller disparity, hidden in the target view) is invalid: a
 * pixel is invalid when some pixel (i, j + k), 0 < k < D, has its target
 * column.  Invalid values are replaced by the nearest valid value of the same
 * row (the smaller one at equal distances); then a 3 x 3 median with
 * replicated borders.  Bit-exact.
 *
 * disp_in      (device) uint8 [B][h][w]; may alias disp_out
 * D            the disparity range of disp_in, 1..256;  w <= 16384
 * disp_out     (device) uint8 [B][h][w]
 * workspace    (device) >= sv_smp_workspace_bytes(B, h, w) bytes, caller-owned
 * Errors: SV_ERR_NULL, SV_ERR_SHAPE, SV_ERR_RANGE, SV_ERR_WORKSPACE.
 */
sv_status sv_smp_median(const uint8_t *disp_in, int B, int h, int w, int D, uint8_t *disp_out,
                        void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Refinement network (Sec. III-B, Table I)                                   */
/* ------------------------------------------------------------------------ */

/*
 * Network shape.  Encoder: three 3x3 stride-2 convolutions 2 -> c1 -> c2 -> c3
 * with leaky ReLU (slope 0.1); head: 1x1 conv c3 -> 2*latent = [mu | logvar];
 * decoder: G3 = 1x1 conv latent -> c3, then three levels that bilinearly
 * resize the previous map to the next encoder level (half-pixel centres),
 * concatenate that level's encoder map (skip connection) and apply a 3x3
 * conv (c3+c2 -> c2, c2+c1 -> c1, c1+2 -> c1); final layer: resize
 * [G0, x0] to H x W and apply a 3x3 conv to one channel, added to the
 * bilinear upscaling of the coarse map.  Input x0 = [f*d/256, I/256] and
 * the output is scaled back by 256 (Sec. III-B2), in full-resolution pixels.
 *
 * Canonical parameter vector (FP32): per layer in the order E1, E2, E3, HEAD,
 * G3, G2, G1, G0, F, the weights in OIHW order followed by the bias.
 */
typedef struct sv_vae_desc {
    int32_t c1, c2, c3; /* encoder widths, each a multiple of 8, <= 256 */
    int32_t latent;     /* latent channels L, multiple of 8, <= 256 */
    int32_t factor;     /* reduction factor f between the pair and the coarse map, 1..8 */
    int32_t dtype;      /* SV_F32, SV_BF16 or SV_F16 */
} sv_vae_desc;

/* Number of FP32 values in the canonical parameter vector (negative on error). */
int64_t sv_vae_param_count(const sv_vae_desc *desc);

/* Bytes of the packed device weight image that sv_vae_pack_weights writes. */
size_t sv_vae_packed_bytes(const sv_vae_desc *desc);

/*
 * Pack the canonical FP32 parameters into the kernels' layout and precision.
 * params (device) float [sv_vae_param_count]; packed_out (device)
 * [sv_vae_packed_bytes], 256-byte aligned.
 */
sv_status sv_vae_pack_weights(const sv_vae_desc *desc, const float *params, void *packed_out,
                              void *stream);

/* Workspace bytes sv_vae_forward / sv_vae_backward need for a batch of B pairs
 * of full resolution H x W (0 on invalid input). */
size_t sv_vae_workspace_bytes(const sv_vae_desc *desc, int B, int H, int W);

/* Bytes of the activations a training forward saves for sv_vae_backward. */
size_t sv_vae_saved_bytes(const sv_vae_desc *desc, int B, int H, int W);

/*
 * Refine a batch of coarse maps.
 *
 * disp_low (device) uint8 [B][h][w], h = ceil(H/f), w = ceil(W/f), coarse
 *          disparity in reduced-resolution pixels (as from sv_cost_wta)
 * img_low  (device) uint8 [B][h][w], the reduced left image
 * eps      (device, nullable) float [B][h3][w3][latent]: NULL = inference,
 *          z = mu; otherwise training, z = mu + eps * exp(logvar/2)
 *          (Eq. (8) in the standard form), h3/w3 = the size after three
 *          stride-2 halvings (ceil each time)
 * out      (device) float [B][H][W], refined disparity in full-res pixels
 * mu_logvar(device, nullable) float [B][h3][w3][2*latent]
 * saved    (device) [sv_vae_saved_bytes]; required when eps != NULL, else ignored
 * workspace(device) [ws_bytes >= sv_vae_workspace_bytes]
 * Errors: SV_ERR_NULL, SV_ERR_SHAPE, SV_ERR_RANGE, SV_ERR_DTYPE, SV_ERR_WORKSPACE.
 */
sv_status sv_vae_forward(const sv_vae_desc *desc, const void *packed_w, const uint8_t *disp_low,
                         const uint8_t *img_low, int B, int H, int W, const float *eps, float *out,
                         float *mu_logvar, void *saved, void *workspace, size_t ws_bytes,
                         void *stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): sv_vae_forward at
 * inference (eps = NULL) with no workspace argument and no allocation.  Its
 * workspace is a device array of the library, SV_STATIC_SCRATCH_BYTES (32 MiB)
 * on every GPU it runs on, held until the process ends; the first call on a
 * device looks up that device's copy.  Same arguments, layouts and results
 * (bitwise) as sv_vae_forward with eps, saved and workspace omitted, for any
 * compute dtype.  A shape whose inference workspace exceeds the array -- for
 * the 1242x375 network (32-64-128, latent 128, f = 4) batches above 2 --
 * returns SV_ERR_WORKSPACE and enqueues nothing.  Every call on one GPU
 * shares the array: calls that overlap on a device (two streams, two threads)
 * race and corrupt each other's results; order them.
 * Errors: SV_ERR_NULL, SV_ERR_SHAPE, SV_ERR_RANGE, SV_ERR_DTYPE,
 *         SV_ERR_WORKSPACE, SV_ERR_HIP.
 */
#define SV_STATIC_SCRATCH_BYTES (32u << 20)
sv_status sv_vae_forward_static(const sv_vae_desc *desc, const void *packed_w,
                                const uint8_t *disp_low, const uint8_t *img_low, int B, int H,
                                int W, float *out, float *mu_logvar, void *stream);

/*
 * Gradient of  sum(dout * out) + kl_weight * KL  with respect to every
 * parameter, for the training forward whose activations are in `saved`
 * (same desc, B, H, W, eps).  KL is the mean over latent elements of
 * 0.5 * (mu^2 + exp(logvar) - 1 - logvar) (Eq. (11) in the standard form).
 * The encoder is recomputed from x0 (activation checkpointing).
 *
 * dout     (device) float [B][H][W], gradient w.r.t. out (per full-res pixel)
 * dmu_logvar (device, nullable) float [B][h3][w3][2*latent]: an extra
 *          gradient w.r.t. [mu | logvar], added to the KL term's
 * grad_out (device) float [sv_vae_param_count], canonical order, overwritten
 */
sv_status sv_vae_backward(const sv_vae_desc *desc, const void *packed_w, const void *saved,
                          int B, int H, int W, const float *eps, const float *dout,
                          const float *dmu_logvar, float kl_weight, float *grad_out,
                          void *workspace, size_t ws_bytes, void *stream);

/*
 * Training loss (a reading of Eqs. (9)-(11)): mean smooth-L1 (beta = 1 px) of
 * out - gt over n pixels plus kl_weight * mean KL over the n_pix_lat * latent
 * latent elements of mu_logvar (rows of 2*latent FP32: mu then logvar;
 * nullable, then KL = 0).
 * loss_out (device) float[3] = {total, data term, KL}; dout (device, nullable)
 * float [n] = clamp(out - gt, -1, 1) / n.  Partial sums in FP64 over a fixed
 * grid and a fixed tree: the result does not depend on scheduling.
 * workspace (device, 8-byte aligned) >= sv_loss_workspace_bytes().
 */
size_t sv_loss_workspace_bytes(void);
sv_status sv_loss(const float *out, const float *gt, int64_t n, const float *mu_logvar,
                  int64_t n_pix_lat, int latent, float kl_weight, float *loss_out, float *dout,
                  void *workspace, size_t ws_bytes, void *stream);

/*
 * One Adam step on FP32 master weights (Sec. IV-A: beta1 = 0.99,
 * beta2 = 0.999, lr = 5e-4; eps is not given in the paper, 1e-8 is usual):
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * w -= lr * (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).  step >= 1.
 */
sv_status sv_adam_step(float *w, const float *g, float *m, float *v, int64_t n, int step,
                       float lr, float beta1, float beta2, float eps, void *stream);

/* ------------------------------------------------------------------------ */
/* Whole path and batches of uneven pairs                                     */
/* ------------------------------------------------------------------------ */

/* One stereo pair of a batch; all pointers (device). */
typedef struct sv_pair {
    const uint8_t *left;  /* [H][W] */
    const uint8_t *right; /* [H][W] */
    float *out;           /* [H][W] refined disparity, full-res pixels */
    uint8_t *disp_low;    /* nullable: [ceil(H/f)][ceil(W/f)] coarse map written here */
    int32_t H, W;
    int32_t D;            /* reduced-resolution disparity range, 1..256 */
} sv_pair;

typedef struct sv_batch_plan sv_batch_plan;

/*
 * Create a plan that runs up to max_n pairs of sizes up to max_H x max_W and
 * ranges up to max_D through the whole path (census, cost + WTA, network)
 * with one launch per stage over all pairs, captured as one hipGraph and
 * replayed per call.  The plan owns its device buffers and graph.
 * win_w, win_h: census window.  Tile shapes come from the autotune cache when
 * it has an entry for these sizes (see sv_autotune), else from defaults.
 */
sv_status sv_batch_plan_create(const sv_vae_desc *desc, int max_n, int max_H, int max_W,
                               int max_D, int win_w, int win_h, sv_batch_plan **plan);
sv_status sv_batch_plan_destroy(sv_batch_plan *plan);

/* Run n pairs (host array) through the plan on `stream`.  Uses the graph
 * unless the environment sets SV_DISABLE_GRAPH=1 (then: the same launches,
 * eager).  Results are bitwise identical either way.  The pair table is
 * written into the next of four pinned host copies and uploaded on `stream`;
 * the call returns without waiting for the device unless that copy's upload
 * from four calls earlier has not finished.  The plan's device buffers are
 * reused by every call: successive calls on one plan must run on one stream
 * (or be ordered by the caller). */
sv_status sv_stereo_batch(sv_batch_plan *plan, const sv_pair *pairs, int n, const void *packed_w,
                          void *stream);

/*
 * The paper's whole system on n pairs of uneven sizes (Sec. III, Sec. IV-A):
 * per pair, in pair order on `stream`, the reduction of both views
 * (sv_census_pair), the coarse matcher -- ZNCC + SGM (sv_zncc_sgm, Eqs.
 * (1)-(6), the paper's main one) or census + SGM (sv_sgm) --, when `median`
 * is 1 the single matching phase and 3 x 3 median (sv_smp_median, Eq. (7)),
 * and the Table I network (sv_tvae_forward, inference) writing pair.out.
 * The coarse map goes to pair.disp_low when it is non-NULL.  Results are
 * bitwise those of the per-pair calls.  No allocation and no host wait:
 * a call can be captured in a hipGraph and replayed.  The pairs reuse one
 * workspace (device, 256-byte aligned) of sv_paper_batch_workspace_bytes for
 * the largest pair (0 on invalid arguments).  Every argument and pair is
 * checked before the first launch.
 * Errors: SV_ERR_NULL, SV_ERR_SHAPE, SV_ERR_RANGE (factor, window, penalties
 * as sv_sgm / sv_zncc_sgm, D), SV_ERR_DTYPE, SV_ERR_UNSUPPORTED (a ZNCC
 * window without a kernel), SV_ERR_WORKSPACE.
 */
#define SV_MATCH_ZNCC_SGM 0
#define SV_MATCH_CENSUS_SGM 1
typedef struct sv_paper_desc {
    int32_t matcher;        /* SV_MATCH_ZNCC_SGM or SV_MATCH_CENSUS_SGM */
    int32_t factor;         /* reduction factor, 1..8 */
    int32_t win_w, win_h;   /* census / ZNCC window (odd) */
    int32_t P1, P2;         /* SGM penalties */
    int32_t median;         /* 1: single matching phase + 3 x 3 median; 0: the SGM map as it is */
    int32_t dtype;          /* Table I network compute dtype: SV_F32, SV_BF16, SV_F16 */
} sv_paper_desc;
size_t sv_paper_batch_workspace_bytes(const sv_paper_desc *desc, int max_H, int max_W, int max_D);
sv_status sv_paper_batch(const sv_paper_desc *desc, const sv_pair *pairs, int n, const void *packed_w,
                         void *workspace, size_t ws_bytes, void *stream);

/*
 * Time the candidate configurations of every stage for this desc and shape
 * on the current device and store the fastest in the autotune cache (a text
 * file at $SV_AUTOTUNE_CACHE, default ~/.cache/sv_autotune.tsv, one line per
 * gfx arch, dtype, channels, latent, factor, batch and size).  A missing or
 * corrupt cache falls back to defaults.  Allocates and frees its own scratch
 * buffers; synchronises.
 */
sv_status sv_autotune(const sv_vae_desc *desc, int B, int H, int W, int D, int win_w, int win_h);

/* Configuration of network layer `layer` (0..8 in the canonical order) for
 * all later calls: cfg in [0, sv_num_layer_cfgs()), or -1 for the default /
 * autotuned choice.  Process-wide.  A configuration is a tile shape plus a
 * split of the channel reduction into 1..4 parts (cfg = tile + ntiles *
 * (split - 1); sv_conv_cfg_name names both).  Results do not depend on the
 * tile shape.  A split > 1 adds the parts' FP32 partial sums in a fixed
 * order, so results are deterministic per split but differ from the
 * unsplit ones by rounding.  Splits apply to sv_vae_forward only (capped by
 * its workspace); the batch plan and the backward pass run unsplit. */
sv_status sv_set_layer_cfg(int layer, int cfg);
int sv_num_layer_cfgs(void);

/* 1 (the default): an inference pass of sv_vae_forward (eps and saved NULL;
 * compute dtype FP32, BF16 or FP16; c3 and L at most 256, multiples of 16
 * for FP32 and of 32 for 16-bit types) runs the
 * latent head (Table I's latent layer, Eq. (8) with z = mu) and G3 as one
 * kernel over the coarsest level:
 * both are 1x1 convolutions, so a workgroup keeps E3 and then mu of its
 * pixels in LDS.  The results are bitwise those of the two layers run one by
 * one without a split; their tile configurations are then unused and the
 * pair is profiled as stage 5 (stage 7 records nothing).  0: always two
 * launches.  Process-wide.  Errors: SV_ERR_RANGE. */
sv_status sv_set_latent_fusion(int on);

/*
 * Profiling: after sv_profile_enable(max_calls) (1..4096), each of the first
 * max_calls launches of every stage records a hipEvent pair around itself on
 * its stream.  Stages: 0 census, 1 cost + WTA, then the network's launches
 * 2 E1, 3 E2, 4 E3, 5 HEAD (with G3 when fused, see sv_set_latent_fusion),
 * 6 reparameterisation (training), 7 G3, 8 G2,
 * 9 G1, 10 G0, 11 (not recorded: the final layer's projection runs inside
 * stage 12), 12 final layer (projection and gather), 13 the second pass
 * (the sum of the partial sums) of every layer that runs a split reduction;
 * the layer's own stage times its first pass alone.
 * sv_profile_read synchronises on the recorded events, writes the summed
 * milliseconds and launch counts of each stage into ms_sum[14] / counts[14]
 * and restarts the counts.  sv_profile_enable(0) disables and frees.
 * sv_profile_repeat(r) (1..64, default 1; errors: SV_ERR_RANGE): while
 * profiling is on, each recorded stage is launched r times back to back
 * between its two events (each launch rewrites the same outputs, so results
 * are unchanged) and counts r launches, so ms_sum / counts is the time of one
 * launch with the cost of the event pair spread over r launches.
 * Process-wide; the library creates and owns the events.
 */
sv_status sv_profile_enable(int max_calls);
sv_status sv_profile_repeat(int repeat);
sv_status sv_profile_read(float *ms_sum, int *counts);

/* The tile configuration (an index, see sv_conv_cfg_name) each of the 9
 * network layers uses for a forward pass of batch B at H x W: an explicit
 * sv_set_layer_cfg override, else the autotune cache entry for this shape,
 * else the default.  cfg_out: (host) int[9]. */
sv_status sv_layer_cfgs(const sv_vae_desc *desc, int B, int H, int W, int *cfg_out);
const char *sv_conv_cfg_name(int cfg);

/* Tile configuration chosen for a stage (for tests and reports):
 * stage 0 = census, 1 = cost+WTA, 2..12 = network layers; writes a short text. */
sv_status sv_tile_config(int stage, char *buf, int buflen);

/* ---- The Table I network as printed (Sec. III-B1) ------------------------------
 *
 * The refinement network in the exact shape of Table I, separate from the
 * configurable network above: feature extraction FE_1 = conv5x5(X_0) and
 * FE_2 = conv5x5(X_1) (32 channels each) on the coarse grid h1 x w1 =
 * ceil(H/f) x ceil(W/f); encoder EN_1 (16, 5x5 stride 2), EN_1_R (8, residual
 * block), EN_2 (32, 5x5 stride 2), EN_2_R (16); a 1x1 head giving one mu and
 * one sigma channel at h3 x w3 (h1 halved twice, rounding up); Eq. (8)
 * z = (mu - 1) + eps * exp(sigma - 1) (eps NULL: z = mu - 1); decoder D_1
 * (32, 1x1 deconvolution), D_1_R (16), D_2 (16, 5x5 stride-2 deconvolution),
 * D_2_R (8), D (16, 5x5 stride-2 deconvolution); and the upsampling layer Y,
 * a 5x5 deconvolution of stride f to one channel at H x W.  Inputs are the
 * "&" concatenations in the table's order; X_0 = f * d / 256 (coarse
 * disparity d), X_1 = I / 256 (reduced left image).  Leaky ReLU (slope 0.1)
 * follows every layer except the head and Y.  A deconvolution has padding 2
 * and its output is cut to the size of the level it feeds (H x W for Y).
 * Output: 256 * Y, disparity in full-resolution px.
 *
 * Parameters: one FP32 vector of sv_tvae_param_count() values, layer by layer
 * in the order FE_1, FE_2, EN_1, EN_1_R, EN_2, EN_2_R, mu&sigma, D_1, D_1_R,
 * D_2, D_2_R, D, Y; each layer's weights [out][in][k][k] (deconvolutions
 * too: y[o][s*i + u - 2][s*j + v - 2] += w[o][c][u][v] * x[c][i][j]), then
 * its bias [out].
 */
int64_t sv_tvae_param_count(void);

/* Bytes of the packed weight image for `dtype` (SV_F32, SV_BF16, SV_F16); 0 if
 * the dtype is invalid. */
size_t sv_tvae_packed_bytes(int dtype);

/*
 * Pack the canonical parameters (device FP32, sv_tvae_param_count() values)
 * into packed_out (device, 256-byte aligned, sv_tvae_packed_bytes(dtype)
 * bytes) in the kernels' layout and precision (the upsampling layer's weights
 * stay FP32 in every dtype).
 * Errors: SV_ERR_NULL, SV_ERR_DTYPE, SV_ERR_RANGE (misaligned packed_out).
 */
sv_status sv_tvae_pack_weights(int dtype, const float *params, void *packed_out, void *stream);

/* Workspace bytes sv_tvae_forward needs for B pairs of full resolution H x W
 * reduced by `factor`; 0 on invalid input. */
size_t sv_tvae_workspace_bytes(int dtype, int factor, int B, int H, int W);

/*
 * Forward pass of the Table I network on B pairs.
 *   disp_low, img_low (device) uint8 [B][h1][w1]: coarse disparity (reduced px)
 *                     and reduced left image, h1 = ceil(H/factor), w1 = ceil(W/factor)
 *   eps       (device, nullable) FP32 [B][h3][w3]: the noise of Eq. (8); NULL = inference
 *   out       (device) FP32 [B][H][W]: disparity in full-resolution px
 *   mu_sigma  (device, nullable) FP32 [B][h3][w3][2]: the head's mu and sigma
 *   workspace (device, 256-byte aligned) >= sv_tvae_workspace_bytes(...)
 * factor in [1, 8]; B * H * W < 2^31; B <= 16383.
 * Errors: SV_ERR_NULL, SV_ERR_DTYPE, SV_ERR_RANGE, SV_ERR_SHAPE, SV_ERR_WORKSPACE.
 */
sv_status sv_tvae_forward(int dtype, int factor, const void *packed_w, const uint8_t *disp_low,
                          const uint8_t *img_low, int B, int H, int W, const float *eps, float *out,
                          float *mu_sigma, void *workspace, size_t ws_bytes, void *stream);

/*
 * The loss of Eqs. (9)-(11) with its gradient.  With N = the number of pixels
 * where occ is set, Loss_1 = (sum over noc of |out - gt| + sum over occ of
 * |out - gt|) / N in px (non-occluded points weigh twice), Loss_2 = 256 *
 * mean over latent positions of 0.5 * ((mu - 1)^2 - 1 + exp(2 (sigma - 1)) -
 * 2 (sigma - 1)), total = Loss_1 + Loss_2 (both already carry the factor 256
 * of Eq. (9): out and gt are in px).
 *   out, gt (device) FP32 [n]; noc, occ (device) uint8 [n] masks (nonzero = set)
 *   mu_sigma (device) FP32 [n_lat][2]
 *   loss_out (device) FP32 [3] = {total, Loss_1, Loss_2}
 *   dout (device, nullable) FP32 [n]: d total / d out (0 where out == gt)
 *   dmu_sigma (device, nullable) FP32 [n_lat][2]: d total / d (mu, sigma)
 *   workspace (device, 8-byte aligned) >= sv_tvae_loss_workspace_bytes()
 * Sums run in FP64 in a fixed order.
 * Errors: SV_ERR_NULL, SV_ERR_SHAPE, SV_ERR_WORKSPACE, SV_ERR_RANGE.
 */
size_t sv_tvae_loss_workspace_bytes(void);
sv_status sv_tvae_loss(const float *out, const float *gt, const uint8_t *noc, const uint8_t *occ,
                       int64_t n, const float *mu_sigma, int64_t n_lat, float *loss_out, float *dout,
                       float *dmu_sigma, void *workspace, size_t ws_bytes, void *stream);

/*
 * Backward pass of the Table I network: the gradient of
 *   sum(dout * out) + sum(dmu_sigma * mu_sigma)
 * with respect to every parameter, in the canonical layout (FP32, overwritten).
 * With dout and dmu_sigma from sv_tvae_loss this is the gradient of the loss
 * of Eqs. (9)-(11).  The forward pass must have run just before on the same
 * inputs, eps and fwd_workspace (its activations are read from there).
 *   disp_low, img_low, eps: as given to sv_tvae_forward (eps nullable)
 *   fwd_workspace (device): the workspace sv_tvae_forward used, unchanged
 *   dout (device) FP32 [B][H][W]; dmu_sigma (device, nullable) FP32 [B][h3][w3][2]
 *   grad_out (device) FP32 [sv_tvae_param_count()]
 *   workspace (device, 256-byte aligned) >= sv_tvae_backward_workspace_bytes(...)
 * Weight gradients are reduced in a fixed order (no floating-point atomics).
 * Errors: SV_ERR_NULL, SV_ERR_DTYPE, SV_ERR_RANGE, SV_ERR_SHAPE, SV_ERR_WORKSPACE.
 */
size_t sv_tvae_backward_workspace_bytes(int dtype, int factor, int B, int H, int W);
sv_status sv_tvae_backward(int dtype, int factor, const void *packed_w, const uint8_t *disp_low,
                           const uint8_t *img_low, int B, int H, int W, const float *eps,
                           const void *fwd_workspace, const float *dout, const float *dmu_sigma,
                           float *grad_out, void *workspace, size_t ws_bytes, void *stream);

/* Tile configuration of launched layer `layer` (0 .. sv_tvae_num_layers()-1:
 * FE, EN_1, EN_1_R, EN_2, EN_2_R, mu&sigma, D_1, D_1_R, D_2, D_2_R, D, Y's tap
 * projection) of sv_tvae_forward, as sv_set_layer_cfg; -1 restores the
 * default.  Results do not depend on the tile shape.  Errors: SV_ERR_RANGE. */
sv_status sv_tvae_set_layer_cfg(int layer, int cfg);
int sv_tvae_num_layers(void);

/* Form of the two stride-2 deconvolutions (D_2, D) in sv_tvae_forward: -1
 * (default) by output size -- four polyphase 3x3 launches (one per output
 * parity class, over the un-inserted input) from 131072 output pixels, else
 * one 5x5 launch over the zero-inserted input; 0 always the zero-inserted
 * form; 1 always polyphase.  Both compute the same deconvolution (they differ
 * in FP32 summation order only).  Errors: SV_ERR_RANGE. */
sv_status sv_tvae_set_deconv_form(int form);

/* Times every tile configuration of each launched layer of sv_tvae_forward
 * alone for this shape (zero weights and inputs; timing does not depend on
 * values), keeps the fastest per layer if the whole pass then runs faster
 * than with the defaults, and uses them for later calls with exactly this
 * (dtype, factor, B, H, W) in this process.  Allocates and frees its own
 * device memory and synchronises the null stream.  Results do not depend on
 * the tile shape (a split changes the FP32 summation order only).
 * Errors: SV_ERR_DTYPE, SV_ERR_RANGE, SV_ERR_SHAPE, SV_ERR_HIP. */
sv_status sv_tvae_autotune(int dtype, int factor, int B, int H, int W);
/* The configuration each launched layer uses for this shape (host int [12]). */
sv_status sv_tvae_layer_cfgs(int dtype, int factor, int B, int H, int W, int *cfg_out);

#ifdef __cplusplus
}
#endif

#endif /* SV_H_ */
