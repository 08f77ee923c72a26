// Internal launcher declarations shared by the host sources of libsv.so.
#pragma once

#include "common.h"

namespace sv {

// ---- batches of uneven pairs ----------------------------------------------------
// A device-resident table describing up to SV_MAXN pairs of different sizes.
// Every stage kernel has a persistent variant that walks the stage's tiles of
// all pairs: tile t belongs to the pair i with cum[stage][i] <= t < cum[stage][i+1].
constexpr int SV_MAXN = 128;
enum BatchStage {
    BS_CENSUS = 0, BS_COST_WTA, BS_E1, BS_E2, BS_E3, BS_HEAD, BS_G3, BS_G2, BS_G1, BS_G0, BS_FPROJ,
    BS_FINAL, BS_NSTAGES
};
struct PairGeo {
    int H, W, D, pad_;
    int h[4], w[4];            // level sizes (level 0 = coarse map)
    long long off[4];          // pixel offset of the pair's level-k maps in the flattened buffers
    const uint8_t *left, *right;
    float *out;                // user's output [H][W]
    uint8_t *disp_out;         // user's coarse map copy, or NULL
};
struct PairTable {
    int n, pad_[3];
    int cum[BS_NSTAGES][SV_MAXN + 1];
    PairGeo pair[SV_MAXN];
};

__device__ __forceinline__ int table_find(const int *cum, int n, int t) {
    int lo = 0, hi = n;  // cum[lo] <= t < cum[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cum[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// ---- matching ----------------------------------------------------------------
sv_status launch_reduce_census(const uint8_t *img0, const uint8_t *img1, int B, int H, int W,
                               int pitch, int f, int win_w, int win_h, uint8_t *low0,
                               uint8_t *low1, uint64_t *cen0, uint64_t *cen1, hipStream_t s);
sv_status launch_cost_wta(const uint64_t *cl, const uint64_t *cr, int B, int h, int w, int D,
                          int nbits, uint8_t *disp, int dsplit, hipStream_t s);
// persistent variants over a pair table (flattened level-0 buffers)
sv_status launch_reduce_census_tab(const PairTable *tab, int grid, int f, int th, int win_w,
                                   int win_h, uint8_t *low0, uint64_t *cen0, uint64_t *cen1,
                                   hipStream_t s);
// census tile height (4 or 16 reduced rows) for a uniform launch of B images
int census_tile_height(int B, int h, int w);
// The windows the ZNCC cost kernel is instantiated for.
bool zncc_window_supported(int win_w, int win_h);
size_t sgm_volume_bytes(int B, int h, int w, int D);
sv_status launch_sgm(const uint64_t *cl, const uint64_t *cr, int B, int h, int w, int D, int nbits,
                     int P1, int P2, uint8_t *vol, uint8_t *disp, hipStream_t s);
sv_status launch_smp_median(const uint8_t *disp, int B, int h, int w, int D, uint8_t *tmp,
                            uint8_t *out, hipStream_t s);
sv_status launch_zncc_cost(const uint8_t *ll, const uint8_t *lr, int B, int h, int w, int D, int Dp,
                           int win_w, int win_h, uint8_t *cost, hipStream_t s);
sv_status launch_zncc_sgm(const uint8_t *ll, const uint8_t *lr, int B, int h, int w, int D, int win_w,
                          int win_h, int P1, int P2, uint8_t *ws, uint8_t *disp, hipStream_t s);
sv_status launch_cost_wta_tab(const PairTable *tab, int grid, const uint64_t *cl, const uint64_t *cr,
                              int nbits, uint8_t *disp, int dsplit, hipStream_t s);
int cost_wta_tile_width(int dsplit);
constexpr int CEN_TILE_W = 64;

// ---- convolution as implicit GEMM ---------------------------------------------
// A convolution input is the channel concatenation of up to two sources.
// SRC_ZINS: the map seen with zeros inserted between its samples (value at
// (y, x) = map[y/2][x/2] for even y and x, else 0), which turns the adjoint
// of a stride-2 convolution into a stride-1 one.
enum SrcKind { SRC_NONE = 0, SRC_TENSOR = 1, SRC_RESIZE = 2, SRC_X0 = 3, SRC_ZINS = 4 };

struct ConvSrc {
    const void *ptr;     // TENSOR / RESIZE: NHWC base; X0: coarse disparity (uint8 [B][h][w])
    const uint8_t *img;  // X0: reduced left image (uint8 [B][h][w])
    int kind;            // SrcKind
    int C;               // channels this source contributes
    int pitch;           // TENSOR / RESIZE: elements per pixel in memory
    int coff;            // TENSOR / RESIZE: first channel within a pixel
    int hs, ws;          // stored spatial size (RESIZE: the smaller map being resized)
    int level;           // pair-table mode: the level whose sizes and offsets apply
    float scale0;        // X0: factor / 256 applied to the disparity channel
    int sdt;             // TENSOR / RESIZE / ZINS storage: 0 = the compute dtype, else 1 + SV_F32/SV_BF16/SV_F16
};

struct ConvParams {
    ConvSrc src[2];
    int B;
    int Hi, Wi;          // input grid (after any resize)
    int Ho, Wo;          // output grid
    int Cin, Cout;
    int cin_pad;         // packed weight row length (Cin rounded up to 8)
    int n_pad;           // packed weight rows (Cout rounded up to 16)
    const void *wpk;     // packed weights [taps][n_pad][cin_pad], compute dtype
    const float *bias;   // [Cout] or NULL
    void *out;           // NHWC output
    int out_pitch, out_coff;
    int act;             // 1: leaky ReLU (slope 0.1)
    int out_f32;         // 1: store FP32 whatever the compute dtype
    // optional epilogue terms of the backward pass, on the output grid:
    const float *add;    // += add[pix * add_pitch + add_coff + n] (FP32)
    int add_pitch, add_coff;
    const void *mask;    // *= (mask[pix * mask_pitch + n] > 0 ? 1 : 0.1), compute dtype
    int mask_pitch;
    // pair-table mode (persistent over the tiles of all pairs); NULL = uniform batch
    const PairTable *tab;
    int stage, in_level, out_level;
    // split reduction (uniform mode only): the input channels are cut into
    // ksplit contiguous ranges of base chunks, each workgroup writes its FP32
    // partial sums to part[(range * B*Ho*Wo + pixel) * n_pad + n], and a second
    // kernel adds the ranges in order and applies the epilogue.  part = NULL
    // disables splitting; part_bytes is its capacity.
    float *part;
    size_t part_bytes;
    int ksplit;
    // INT8 layers: per-row weight scales, and the per-tensor maxima of the
    // sources (amax_in, AMAX_SUB words each: max |value| as FP32 bits, NULL =
    // no source) from which the input scale is formed; any layer with amax_out
    // set records the max |stored value| of its output there (one word of
    // AMAX_SUB per workgroup slot, combined by the reader)
    const float *wscale;
    const uint32_t *amax_in[2];
    uint32_t *amax_out;
    // output phase (uniform launches, never split): 0 = dense output; else
    // output pixel (oy, ox) of this launch is (2 oy + py, 2 ox + px) of a
    // Ho_full x Wo_full map, ophase = 1 + 2 py + px (one parity class of a
    // stride-2 deconvolution)
    int ophase, Ho_full, Wo_full;
    // 1: a split launch leaves its FP32 partials in part for the consumer to
    // add (the fused latent kernel), instead of launching the second pass
    int defer_sum;
    // final-layer projection in the epilogue (G0 at inference; uniform or
    // pair-table launches, never split, one channel tile per workgroup with
    // all of it in each wave): instead of storing the output map y, write
    //   proj_out[t * proj_plane + pix] = sum_c proj_w[t * proj_pitch + c] y_c
    //       + proj_w[t * proj_pitch + Cout] * proj_scale0 * d
    //       + proj_w[t * proj_pitch + Cout + 1] * img / 256
    // for the nine taps t, y_c as it would have been stored (rounded to the
    // storage dtype), d / img the coarse maps at the pixel.  NULL: store y.
    const float *proj_w;
    int proj_pitch;
    float *proj_out;
    long long proj_plane;
    const uint8_t *proj_disp, *proj_img;
    float proj_scale0;
};
constexpr int AMAX_SUB = 64;

// cfg selects the tile shape and the reduction split (see conv.hip); ks = 1, 3
// or 5, stride = 1 or 2 (ks = 1: stride 1 only).
sv_status launch_conv(int dtype, int ks, int stride, int cfg, const ConvParams &p, hipStream_t s);
// launch_conv that also reports the reduction split it used (1: none)
sv_status launch_conv_split(int dtype, int ks, int stride, int cfg, const ConvParams &p, hipStream_t s,
                            int *ksplit_used);
// the second pass of a split reduction (ksplit > 1) of a launch made with
// p.defer_sum set: sums the partials and applies the epilogue; a no-op for 1
sv_status launch_split_sum(int dtype, const ConvParams &p, int ksplit, hipStream_t s);
// persistent launch over p.tab's tiles of stage p.stage with `grid` workgroups
sv_status launch_conv_tab(int dtype, int ks, int stride, int cfg, const ConvParams &p, int grid,
                          hipStream_t s);
void conv_cfg_tile(int cfg, int &TH, int &TN);
// cfg, or the fallback tile shape (same split) when cfg's tile does not fit
// the LDS for this kernel size and stride; launches resolve the same way
int conv_resolve_cfg(int dtype, int ks, int stride, int cfg);
int conv_num_tiles();  // tile shapes; cfg = tile + conv_num_tiles() * (ksplit - 1)
constexpr int CONV_MAX_SPLIT = 4;
// the split a launch of configuration cfg actually uses (1 when it cannot split)
int conv_effective_split(int dtype, int cfg, int Cin, long long npix, int n_pad, const float *part,
                         size_t part_bytes);
// partial-sum buffer of a split launch: at most this many bytes per forward pass
constexpr size_t CONV_PART_CAP = (size_t)16 << 20;
int conv_num_cfgs();
const char *conv_cfg_name(int cfg);

// Packs canonical OIHW FP32 weights of one layer into [taps][n_pad][cin_pad].
// mode 0: forward rows = output channels; mode 1 (final layer): taps = 1 and
// row t = source tap t; mode 2: adjoint, rows = input channels, columns =
// output channels, kernel flipped.
sv_status launch_pack(int dtype, const float *w, int Cout, int Cin, int k, int n_pad, int cin_pad,
                      int mode, void *dst, hipStream_t s);
// INT8 forward packing: codes [taps][n_pad][cin_pad] and the per-row scales
// (FP32 [n_pad], 0 past Cout)
sv_status launch_pack_i8(const float *w, int Cout, int Cin, int k, int n_pad, int cin_pad, int8_t *dst,
                         float *scale, hipStream_t s);
// Weight-gradient partial sums of one layer (the backward's k_wgrad, kernel
// sizes 1, 3, 5): part[split][o_pad][taps][cinp] then the bias partials
// part_b[split][o_pad]; dy is the output gradient (FP32 NHWC, pitch dy_pitch).
struct WgradShape { int splits, o_pad, taps, cinp; };
size_t wgrad_partial_floats(int B, int Ho, int Wo, int Cin, int Cout, int ks);
sv_status launch_wgrad_partials(int dtype, int ks, int stride, ConvSrc s0, ConvSrc s1, int B, int Hi, int Wi,
                                int Ho, int Wo, int Cout, const float *dy, int dy_pitch, float *part,
                                WgradShape &shape, hipStream_t st);

// INT8 pass prologue: zero nslots * AMAX_SUB words, then record the amax of
// x0 = [scale0 * d, img / 256] over n coarse pixels in slot x0_slot
sv_status launch_amax_prologue(uint32_t *amax, int nslots, int x0_slot, const uint8_t *disp,
                               const uint8_t *img, long long n, float scale0, hipStream_t s);

// The grid of a persistent launch of fn (256 threads, dyn_lds bytes of
// dynamic LDS) that wants `want` workgroups: at most what the current device
// holds at once.  Host-side queries only (cached per device, kernel and LDS
// size), nothing is enqueued, so it may run during stream capture.
long long resident_grid(const void *fn, size_t dyn_lds, long long want);

// storage dtype code of a source (see ConvSrc::sdt)
constexpr int SDT_SAME = 0, SDT_F32 = 1 + SV_F32, SDT_BF16 = 1 + SV_BF16, SDT_F16 = 1 + SV_F16;

// The first encoder layer (3x3, stride 2, two input channels x0 = [scale0 * d,
// img / 256], leaky ReLU) as a direct stencil, FP32 arithmetic, output NHWC
// [B][h1][w1][c1] in the compute dtype (SV_F32, SV_BF16, SV_F16); weights
// packed [9][n_pad][cin_pad] in that dtype, FP32 bias.  c1: multiple of 8, <= 256.
// SV_I8: INT8 weight codes with per-channel scales wscale, x0 quantised with
// the scale from its recorded maxima amax_in (AMAX_SUB words), exact integer
// sums, BF16 output, its max |value| recorded in amax_out (all three required).
sv_status launch_enc1(int dtype, const uint8_t *disp, const uint8_t *img, float scale0, int B, int h0, int w0,
                      int h1, int w1, int c1, const void *wpk, int n_pad, int cin_pad, const float *bias,
                      void *out, hipStream_t st, const float *wscale = nullptr,
                      const uint32_t *amax_in = nullptr, uint32_t *amax_out = nullptr);
// persistent variant over the pair table (stage BS_E1; level-0 inputs, level-1 output)
sv_status launch_enc1_tab(int dtype, const PairTable *tab, int grid, const uint8_t *disp, const uint8_t *img,
                          float scale0, int c1, const void *wpk, int n_pad, int cin_pad, const float *bias,
                          void *out, hipStream_t st);
int enc1_tiles(int h1, int w1);

// ---- network glue ---------------------------------------------------------------
// The final layer from the coarse maps: with T[t] = W_F[t] . [G0, x0] (FP32
// weights [9][wf_pitch], x0 = [f * d / 256, img / 256]),
// out[b][Y][X] = 256 * (bias + sum_taps resize(T[tap])(Y+u-1, X+v-1) + resize(f*d/256)(Y, X)).
// G0: NHWC [B][h][w][c1] in dtype; disp, img: uint8 [B][h][w].
// Inference: the latent head (ph, [mu | logvar] in FP32) and G3 (pg, reading
// mu) as one kernel over npix pixels of the coarsest level; same bits as the
// two layers launched one by one, unsplit.  latent_fusable tells whether the
// widths allow it (whole base chunks, at most 256 channels).
bool latent_fusable(int dtype, int c3, int L);
// e3part / e3split / e3bias: when E3 ran split with its sum deferred, its
// FP32 partials (ranges in order), which the kernel adds, biases and passes
// through the leaky ReLU as the second pass would (E3 itself is then never
// stored); e3split <= 1 reads the stored E3.
sv_status launch_latent(int dtype, const ConvParams &ph, const ConvParams &pg, int npix,
                        const float *e3part, int e3split, const float *e3bias, hipStream_t st);
// The final layer from precomputed tap projections T (FP32 [9][plane], plane
// = pixels of the coarse maps; written by G0's epilogue, ConvParams::proj_*):
// the gather and the residual base of launch_final without the projection.
// Output rows per tile of the final gather at factor f for a launch over
// out_px output pixels (tiles are FIN_TILE_W wide): 16, 32 or 64.
int gather_tile_h(int f, long long out_px);
sv_status launch_final_gather(const float *T, long long plane, const uint8_t *disp, int f,
                              const float *biasF, int B, int h, int w, int H, int W, float *out,
                              hipStream_t s);
sv_status launch_final_gather_tab(const PairTable *tab, int grid, const float *T, long long plane,
                                  const uint8_t *disp, int f, int th, const float *biasF, hipStream_t s);
// whether a conv tile configuration can carry the projection epilogue for a
// layer with cout output channels (one channel tile, all of it in each wave)
bool conv_cfg_projects(int cfg, int cout);
// the configuration a persistent pair-table launch runs for cfg
int conv_persistent_cfg(int cfg);
sv_status launch_final(int dtype, const void *G0, int c1, const uint8_t *disp, const uint8_t *img,
                       const float *wF, int wf_pitch, int f, const float *biasF, int B, int h,
                       int w, int H, int W, float *out, hipStream_t s);
sv_status launch_final_tab(const PairTable *tab, int grid, int dtype, const void *G0, int c1,
                           const uint8_t *disp, const uint8_t *img, const float *wF, int wf_pitch,
                           int f, const float *biasF, hipStream_t s);
constexpr int FIN_TILE_W = 64, FIN_TILE_H = 16;
sv_status launch_reparam(const float *ml, const float *eps, int npix, int L, void *z, int dtype,
                         hipStream_t s);

}  // namespace sv
