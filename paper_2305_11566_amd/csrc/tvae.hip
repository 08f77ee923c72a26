// The refinement network exactly in the shape of Table I (Sec. III-B1):
// feature extraction, encoder with residual blocks, the one-channel mu /
// sigma head with the shifts of Eq. (8), decoder with 5x5 stride-2
// deconvolutions and skip connections, and the final upsampling layer; plus
// the loss of Eqs. (9)-(11).
//
// Layout: each level keeps one NHWC map whose channel ranges are the maps the
// table concatenates, in the table's order, so every "A & B & C" input is one
// contiguous channel range read by one convolution source:
//   level 1 (h1 x w1 = the coarse map): [D 16 | FE_1 32 | FE_2 32]        80 ch
//   level 2 (h1/2):                     [D_2 16 | EN_1 16 | EN_1_R 8 | D_2_R 8] 48 ch
//   level 3 (h1/4):                     [D_1 32 | EN_2 32 | EN_2_R 16 | D_1_R 16] 96 ch
// A stride-2 deconvolution is a stride-1 convolution with the flipped kernel
// over its input seen with zeros inserted between samples (SRC_ZINS), cut to
// the size of the level it feeds.  FE_1 and FE_2 run as one layer over the two
// input channels with block-diagonal weights.  The final upsampling layer
// (5x5, stride f, one output channel) runs as a 1x1 projection of the level-1
// map and X_0 onto its 25 taps (MFMA), then a gather that adds, for each
// full-resolution pixel, the taps that land on it.
#include <algorithm>
#include <array>
#include <atomic>
#include <initializer_list>
#include <map>
#include <mutex>
#include <tuple>

#include "kernels.h"

namespace sv {

namespace {

#define SV_TRY_STATUS(x)            \
    do {                            \
        sv_status r_ = (x);         \
        if (r_ != SV_OK) return r_; \
    } while (0)

constexpr int TV_K = 5, TV_TAPS = 25;
constexpr int L1C = 80, L2C = 48, L3C = 96, ZC = 8, TC = 32;

// canonical layers, in the table's order: weights [out][in][k][k], then bias
struct CanonLayer { int cout, cin, k; };
constexpr CanonLayer kCanon[] = {
    {32, 1, 5},   // FE_1
    {32, 1, 5},   // FE_2
    {16, 64, 5},  // EN_1
    {8, 16, 5},   // EN_1_R
    {32, 24, 5},  // EN_2
    {16, 32, 5},  // EN_2_R
    {2, 48, 1},   // mu & sigma
    {32, 1, 1},   // D_1 (1x1 deconvolution)
    {16, 80, 5},  // D_1_R
    {16, 96, 5},  // D_2 (deconvolution, stride 2)
    {8, 40, 5},   // D_2_R
    {16, 48, 5},  // D (deconvolution, stride 2)
    {1, 81, 5},   // Y (upsampling layer, stride f)
};
constexpr int NCANON = 13;
enum { C_FE1 = 0, C_FE2, C_EN1, C_EN1R, C_EN2, C_EN2R, C_MS, C_D1, C_D1R, C_D2, C_D2R, C_D, C_Y };

// launched layers (FE_1 and FE_2 fused; Y as its tap projection)
enum { T_FE = 0, T_EN1, T_EN1R, T_EN2, T_EN2R, T_MS, T_D1, T_D1R, T_D2, T_D2R, T_D, T_YP, T_NL };
struct TvLayer { int cout, cin, k, stride; };  // stride of the launched convolution
constexpr TvLayer kLayers[T_NL] = {
    {64, 2, 5, 1}, {16, 64, 5, 2}, {8, 16, 5, 1}, {32, 24, 5, 2}, {16, 32, 5, 1}, {2, 48, 1, 1},
    {32, 1, 1, 1}, {16, 80, 5, 1}, {16, 96, 5, 1}, {8, 40, 5, 1}, {16, 48, 5, 1}, {TV_TAPS, 82, 1, 1},
};

int64_t canon_off(int i) {
    int64_t o = 0;
    for (int j = 0; j < i; ++j) o += (int64_t)kCanon[j].cout * kCanon[j].cin * kCanon[j].k * kCanon[j].k + kCanon[j].cout;
    return o;
}

inline int rup(int v, int m) { return (v + m - 1) / m * m; }

struct TvShape {
    int dtype, es;
    int n_pad[T_NL], cin_pad[T_NL];
    size_t w_off[T_NL], b_off[T_NL], bytes;
    // adjoint packs of the input gradient: rows = the layer's inputs (Y's
    // projection: the 80 level-1 channels), columns = its outputs; 0 for FE
    int bn_pad[T_NL], bcin_pad[T_NL];
    size_t bw_off[T_NL];
    // stride-2 deconvolutions (D_2, D) in polyphase form: per output parity
    // class a 3x3 kernel [9][n_pad][cin_pad] over the un-inserted input
    size_t ph_off[T_NL][4];
};

// Launched layers' input rows of the adjoint pack (0: no input gradient).
constexpr int kAdjRows[T_NL] = {0, 64, 16, 24, 32, 48, 1, 80, 96, 40, 48, 80};

TvShape tv_shape(int dtype) {
    TvShape s{};
    s.dtype = dtype;
    s.es = dtype_bytes(dtype);
    size_t off = 0;
    for (int i = 0; i < T_NL; ++i) {
        const TvLayer &l = kLayers[i];
        s.n_pad[i] = rup(l.cout, 16);
        s.cin_pad[i] = rup(l.cin, 8);
        // the tap projection stays FP32 in every mode, like the other network's
        // final layer: its few weights dominate the reduced-precision error
        const int les = i == T_YP ? 4 : s.es;
        s.w_off[i] = off;
        off = align256(off + (size_t)l.k * l.k * s.n_pad[i] * s.cin_pad[i] * les);
        s.b_off[i] = off;
        off = align256(off + (size_t)s.n_pad[i] * sizeof(float));
    }
    for (int i = 0; i < T_NL; ++i) {
        s.bw_off[i] = 0;
        s.bn_pad[i] = s.bcin_pad[i] = 0;
        if (!kAdjRows[i]) continue;
        s.bn_pad[i] = rup(kAdjRows[i], 16);
        s.bcin_pad[i] = rup(kLayers[i].cout, 8);
        const int les = i == T_YP ? 4 : s.es;
        s.bw_off[i] = off;
        off = align256(off + (size_t)kLayers[i].k * kLayers[i].k * s.bn_pad[i] * s.bcin_pad[i] * les);
    }
    for (int i = 0; i < T_NL; ++i)
        for (int ph = 0; ph < 4; ++ph) {
            s.ph_off[i][ph] = 0;
            if (i != T_D2 && i != T_D) continue;
            s.ph_off[i][ph] = off;
            off = align256(off + (size_t)9 * s.n_pad[i] * s.cin_pad[i] * s.es);
        }
    s.bytes = off;
    return s;
}

struct TvLevels { int H, W, h[4], w[4]; };  // h[1..3]: levels 1..3

TvLevels tv_levels(int f, int H, int W) {
    TvLevels lv{};
    lv.H = H; lv.W = W;
    lv.h[1] = cdiv(H, f); lv.w[1] = cdiv(W, f);
    for (int k = 2; k < 4; ++k) { lv.h[k] = cdiv(lv.h[k - 1], 2); lv.w[k] = cdiv(lv.w[k - 1], 2); }
    return lv;
}

struct TvAct { size_t L1, L2, L3, Z, ML, T, part, part_bytes, total; };

// output level of each launched layer
constexpr int kOutLevel[T_NL] = {1, 2, 2, 3, 3, 3, 3, 3, 2, 2, 1, 1};

TvAct tv_act(int es, const TvLevels &lv, int B) {
    auto px = [&](int k) { return (size_t)B * lv.h[k] * lv.w[k]; };
    TvAct a{};
    size_t o = 0;
    // partial sums of split-reduction launches (small grids): room for the
    // largest layer output at the maximum split, capped
    size_t part = 0;
    for (int i = 0; i < T_NL; ++i)
        part = std::max(part, (size_t)CONV_MAX_SPLIT * px(kOutLevel[i]) * rup(kLayers[i].cout, 16) * sizeof(float));
    a.part_bytes = std::min(part, CONV_PART_CAP);
    a.L1 = o; o = align256(o + px(1) * L1C * es);
    a.L2 = o; o = align256(o + px(2) * L2C * es);
    a.L3 = o; o = align256(o + px(3) * L3C * es);
    a.Z = o;  o = align256(o + px(3) * ZC * es);
    a.ML = o; o = align256(o + px(3) * 2 * sizeof(float));
    a.T = o;  o = align256(o + px(1) * TC * sizeof(float));
    a.part = o; o = align256(o + a.part_bytes);
    a.total = o;
    return a;
}

std::atomic<int> g_tv_cfg[T_NL];
struct TvCfgInit {
    TvCfgInit() { for (auto &v : g_tv_cfg) v.store(-1); }
} g_tv_cfg_init;

// Configurations sv_tvae_autotune chose, per (dtype, factor, B, H, W), for
// this process.
std::mutex g_tv_mu;
std::map<std::tuple<int, int, int, int, int>, std::array<int, T_NL>> g_tv_tuned;

// Default: tile th4_tn16 / th4_tn32 by output width; grids of fewer than 256
// workgroups (the coarse levels of small batches) split the reduction over
// up to four channel ranges so that more CUs take part.
int tv_heuristic_cfg(int layer, int B, int Ho, int Wo) {
    const int tn = kLayers[layer].cout <= 16 ? 16 : 32;
    const int tile = tn == 16 ? 5 /* th4_tn16 */ : 2 /* th4_tn32 */;
    const long long nwg = (long long)cdiv(Wo, 16) * cdiv(Ho, 4) * B * cdiv(kLayers[layer].cout, tn);
    int split = 1;
    while (split < CONV_MAX_SPLIT && nwg * split < 256) ++split;
    return tile + conv_num_tiles() * (split - 1);
}

// Per launched layer: an explicit override, else the tuned choice for this
// shape, else the heuristic.
void tv_layer_cfgs(int dtype, int f, int B, int H, int W, int *cfg) {
    const TvLevels lv = tv_levels(f, H, W);
    std::array<int, T_NL> tuned{};
    bool have = false;
    {
        std::lock_guard<std::mutex> g(g_tv_mu);
        auto it = g_tv_tuned.find(std::make_tuple(dtype, f, B, H, W));
        if (it != g_tv_tuned.end()) { tuned = it->second; have = true; }
    }
    for (int i = 0; i < T_NL; ++i) {
        const int ov = g_tv_cfg[i].load();
        const int k = kOutLevel[i];
        cfg[i] = (ov >= 0 && ov < conv_num_cfgs()) ? ov : (have ? tuned[i] : tv_heuristic_cfg(i, B, lv.h[k], lv.w[k]));
    }
}

// ---- packing ------------------------------------------------------------------------
// One job writes the rows [row0, row0 + cout) of a packed layer from one
// canonical layer: column c of the packed row reads canonical input channel
// cmap[c] (-1: zero); flip turns a deconvolution into the equivalent
// correlation over the zero-inserted input; proj packs the upsampling layer as
// one row per tap.
struct PackJob {
    const float *w;   // canonical weights of the layer
    int cout, cin, k, row0, taps, n_pad, cin_pad, flip, proj;
    int cmap[96];
};

template <int DT>
__global__ void k_tv_pack_t(const PackJob j, typename Elem<DT>::T *__restrict__ dst) {
    const int rows = j.proj ? TV_TAPS : j.cout;
    const int total = j.taps * rows * j.cin_pad;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int c = e % j.cin_pad;
        const int r = (e / j.cin_pad) % rows;
        const int tap = e / (j.cin_pad * rows);
        const int ci = c < 96 ? j.cmap[c] : -1;
        float v = 0.f;
        if (ci >= 0) {
            if (j.proj) v = j.w[(size_t)ci * j.k * j.k + r];  // output channel 0, tap r
            else v = j.w[((size_t)r * j.cin + ci) * j.k * j.k + (j.flip ? j.k * j.k - 1 - tap : tap)];
        }
        dst[((size_t)tap * j.n_pad + j.row0 + r) * j.cin_pad + c] = Elem<DT>::make(v);
    }
}

// Adjoint pack of one launched layer: dst[tap][n][c] with n over the layer's
// inputs (canonical input channel rmap[n]) and c over its outputs.  A
// convolution's input gradient correlates the output gradient with the
// flipped kernel (over the zero-inserted gradient for stride 2); a
// deconvolution's is the stride-2 correlation with the kernel as it is; proj:
// the upsampling layer, one column per tap.
struct AdjJob {
    const float *w;
    int cout, cin, k, rows, cols, taps, n_pad, cin_pad, flip, proj;
    int rmap[96];
};

template <int DT>
__global__ void k_tv_pack_adj(const AdjJob j, typename Elem<DT>::T *__restrict__ dst) {
    const int total = j.taps * j.n_pad * j.cin_pad;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int c = e % j.cin_pad;
        const int n = (e / j.cin_pad) % j.n_pad;
        const int tap = e / (j.cin_pad * j.n_pad);
        float v = 0.f;
        const int ci = n < j.rows ? j.rmap[n] : -1;
        if (ci >= 0 && c < j.cols) {
            if (j.proj) v = j.w[(size_t)ci * j.k * j.k + c];  // output channel 0, tap c
            else v = j.w[((size_t)c * j.cin + ci) * j.k * j.k + (j.flip ? j.k * j.k - 1 - tap : tap)];
        }
        dst[e] = Elem<DT>::make(v);
    }
}

// One parity class (py, px) of a stride-2, padding-2 5x5 deconvolution as a
// 3x3, padding-1 correlation over the un-inserted input: output 2a + py takes
// input row a - 1 + t with the weight row u = py + 4 - 2t (none outside 0..4),
// and likewise for columns.
template <int DT>
__global__ void k_tv_pack_phase(const float *__restrict__ w, int cout, int cin, int n_pad, int cin_pad, int py,
                                int px, typename Elem<DT>::T *__restrict__ dst) {
    const int total = 9 * n_pad * cin_pad;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int c = e % cin_pad;
        const int o = (e / cin_pad) % n_pad;
        const int tap = e / (cin_pad * n_pad);
        const int u = py + 4 - 2 * (tap / 3), v = px + 4 - 2 * (tap % 3);
        float val = 0.f;
        if (o < cout && c < cin && u >= 0 && u < TV_K && v >= 0 && v < TV_K)
            val = w[(((size_t)o * cin + c) * TV_K + u) * TV_K + v];
        dst[e] = Elem<DT>::make(val);
    }
}

__global__ void k_zero_bytes(uint32_t *__restrict__ p, size_t n_words) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n_words; e += (size_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

__global__ void k_tv_bias(const float *__restrict__ b, int n, float *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = b[i];
}

sv_status run_pack_job(int dt, const PackJob &j, void *dst, hipStream_t st) {
    const int rows = j.proj ? TV_TAPS : j.cout;
    const int total = j.taps * rows * j.cin_pad;
    const int blocks = std::min((total + 255) / 256, 1024);
    switch (dt) {
    case SV_F32: hipLaunchKernelGGL(k_tv_pack_t<SV_F32>, dim3(blocks), dim3(256), 0, st, j, (float *)dst); break;
    case SV_BF16: hipLaunchKernelGGL(k_tv_pack_t<SV_BF16>, dim3(blocks), dim3(256), 0, st, j, (uint16_t *)dst); break;
    case SV_F16: hipLaunchKernelGGL(k_tv_pack_t<SV_F16>, dim3(blocks), dim3(256), 0, st, j, (uint16_t *)dst); break;
    default: return SV_ERR_DTYPE;
    }
    SV_LAUNCH_CHECK("k_tv_pack");
    return SV_OK;
}

sv_status tv_pack(const TvShape &s, const float *params, void *packed, hipStream_t st) {
    // zero padding rows and columns first (a fill kernel, not a memset node)
    const size_t words = s.bytes / 4;
    hipLaunchKernelGGL(k_zero_bytes, dim3((unsigned)std::min<size_t>((words + 255) / 256, 4096)), dim3(256), 0, st,
                       (uint32_t *)packed, words);
    SV_LAUNCH_CHECK("k_zero_bytes");
    char *P = (char *)packed;
    auto job = [&](int canon, int layer, int row0, bool flip, auto colmap) -> sv_status {
        PackJob j{};
        const CanonLayer &c = kCanon[canon];
        j.w = params + canon_off(canon);
        j.cout = c.cout; j.cin = c.cin; j.k = c.k; j.row0 = row0;
        j.proj = layer == T_YP;
        j.taps = j.proj ? 1 : c.k * c.k;
        j.n_pad = s.n_pad[layer]; j.cin_pad = s.cin_pad[layer];
        j.flip = flip;
        for (int q = 0; q < 96; ++q) j.cmap[q] = q < j.cin_pad ? colmap(q) : -1;
        SV_TRY_STATUS(run_pack_job(layer == T_YP ? SV_F32 : s.dtype, j, P + s.w_off[layer], st));
        // bias of these rows (the projection has none: the gather adds Y's bias)
        if (!j.proj) {
            hipLaunchKernelGGL(k_tv_bias, dim3(1), dim3(64), 0, st, j.w + (size_t)c.cout * c.cin * c.k * c.k, c.cout,
                               (float *)(P + s.b_off[layer]) + row0);
            SV_LAUNCH_CHECK("k_tv_bias");
        }
        return SV_OK;
    };
    auto ident = [](int cin) { return [cin](int q) { return q < cin ? q : -1; }; };
    // FE: rows 0..31 read channel 0 (X_0), rows 32..63 channel 1 (X_1)
    SV_TRY_STATUS(job(C_FE1, T_FE, 0, false, [](int q) { return q == 0 ? 0 : -1; }));
    SV_TRY_STATUS(job(C_FE2, T_FE, 32, false, [](int q) { return q == 1 ? 0 : -1; }));
    SV_TRY_STATUS(job(C_EN1, T_EN1, 0, false, ident(64)));
    SV_TRY_STATUS(job(C_EN1R, T_EN1R, 0, false, ident(16)));
    SV_TRY_STATUS(job(C_EN2, T_EN2, 0, false, ident(24)));
    SV_TRY_STATUS(job(C_EN2R, T_EN2R, 0, false, ident(32)));
    SV_TRY_STATUS(job(C_MS, T_MS, 0, false, ident(48)));
    SV_TRY_STATUS(job(C_D1, T_D1, 0, false, ident(1)));
    SV_TRY_STATUS(job(C_D1R, T_D1R, 0, false, ident(80)));
    SV_TRY_STATUS(job(C_D2, T_D2, 0, true, ident(96)));
    SV_TRY_STATUS(job(C_D2R, T_D2R, 0, false, ident(40)));
    SV_TRY_STATUS(job(C_D, T_D, 0, true, ident(48)));
    // projection columns: the level-1 map [D | FE_1 | FE_2], then X_0, X_1;
    // the table's order is D & X_0 & FE_1 & FE_2 (X_1 does not enter)
    SV_TRY_STATUS(job(C_Y, T_YP, 0, false, [](int q) { return q < 16 ? q : (q < 80 ? q + 1 : (q == 80 ? 16 : -1)); }));
    // Y's bias goes to the projection's bias slot, read by the gather
    hipLaunchKernelGGL(k_tv_bias, dim3(1), dim3(64), 0, st, params + canon_off(C_Y) + 81 * 25, 1,
                       (float *)(P + s.b_off[T_YP]));
    SV_LAUNCH_CHECK("k_tv_bias");
    // polyphase packs of the stride-2 deconvolutions
    for (int li : {T_D2, T_D}) {
        const int canon = li == T_D2 ? C_D2 : C_D;
        const CanonLayer &c = kCanon[canon];
        for (int ph = 0; ph < 4; ++ph) {
            const int total = 9 * s.n_pad[li] * s.cin_pad[li];
            const int blocks = std::min((total + 255) / 256, 1024);
            void *dst = P + s.ph_off[li][ph];
            const float *w = params + canon_off(canon);
            switch (s.dtype) {
            case SV_F32: hipLaunchKernelGGL(k_tv_pack_phase<SV_F32>, dim3(blocks), dim3(256), 0, st, w, c.cout, c.cin, s.n_pad[li], s.cin_pad[li], ph >> 1, ph & 1, (float *)dst); break;
            case SV_BF16: hipLaunchKernelGGL(k_tv_pack_phase<SV_BF16>, dim3(blocks), dim3(256), 0, st, w, c.cout, c.cin, s.n_pad[li], s.cin_pad[li], ph >> 1, ph & 1, (uint16_t *)dst); break;
            default: hipLaunchKernelGGL(k_tv_pack_phase<SV_F16>, dim3(blocks), dim3(256), 0, st, w, c.cout, c.cin, s.n_pad[li], s.cin_pad[li], ph >> 1, ph & 1, (uint16_t *)dst); break;
            }
            SV_LAUNCH_CHECK("k_tv_pack_phase");
        }
    }
    // adjoint packs (the backward pass)
    auto adj = [&](int canon, int layer, bool flip, auto rowmap) -> sv_status {
        AdjJob j{};
        const CanonLayer &c = kCanon[canon];
        j.w = params + canon_off(canon);
        j.cout = c.cout; j.cin = c.cin; j.k = c.k;
        j.proj = layer == T_YP;
        j.rows = kAdjRows[layer];
        j.cols = kLayers[layer].cout;
        j.taps = kLayers[layer].k * kLayers[layer].k;
        j.n_pad = s.bn_pad[layer]; j.cin_pad = s.bcin_pad[layer];
        j.flip = flip;
        for (int q = 0; q < 96; ++q) j.rmap[q] = q < j.rows ? rowmap(q) : -1;
        const int total = j.taps * j.n_pad * j.cin_pad;
        const int blocks = std::min((total + 255) / 256, 1024);
        void *dst = P + s.bw_off[layer];
        switch (layer == T_YP ? SV_F32 : s.dtype) {
        case SV_F32: hipLaunchKernelGGL(k_tv_pack_adj<SV_F32>, dim3(blocks), dim3(256), 0, st, j, (float *)dst); break;
        case SV_BF16: hipLaunchKernelGGL(k_tv_pack_adj<SV_BF16>, dim3(blocks), dim3(256), 0, st, j, (uint16_t *)dst); break;
        default: hipLaunchKernelGGL(k_tv_pack_adj<SV_F16>, dim3(blocks), dim3(256), 0, st, j, (uint16_t *)dst); break;
        }
        SV_LAUNCH_CHECK("k_tv_pack_adj");
        return SV_OK;
    };
    auto idr = [](int q) { return q; };
    SV_TRY_STATUS(adj(C_EN1, T_EN1, true, idr));
    SV_TRY_STATUS(adj(C_EN1R, T_EN1R, true, idr));
    SV_TRY_STATUS(adj(C_EN2, T_EN2, true, idr));
    SV_TRY_STATUS(adj(C_EN2R, T_EN2R, true, idr));
    SV_TRY_STATUS(adj(C_MS, T_MS, false, idr));
    SV_TRY_STATUS(adj(C_D1, T_D1, false, idr));
    SV_TRY_STATUS(adj(C_D1R, T_D1R, true, idr));
    SV_TRY_STATUS(adj(C_D2, T_D2, false, idr));
    SV_TRY_STATUS(adj(C_D2R, T_D2R, true, idr));
    SV_TRY_STATUS(adj(C_D, T_D, false, idr));
    // the upsampling layer's rows: the level-1 channels [D | FE_1 | FE_2] in the
    // table's order D & X_0 & FE_1 & FE_2 (X_0 needs no gradient)
    SV_TRY_STATUS(adj(C_Y, T_YP, false, [](int q) { return q < 16 ? q : q + 1; }));
    return SV_OK;
}

// ---- Eq. (8) and the final gather ------------------------------------------------
// z = (mu - 1) + eps * exp(sigma - 1) (eps NULL: z = mu - 1), stored as channel 0
// of an 8-channel row (channels 1..7 zero) so that the 1x1 deconvolution reads
// whole channel groups.
template <int DT>
__global__ void k_tv_reparam(const float *__restrict__ ml, const float *__restrict__ eps, int n,
                             typename Elem<DT>::T *__restrict__ z) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = ml[2 * i] - 1.0f;
    if (eps) v += eps[i] * expf(ml[2 * i + 1] - 1.0f);
    typename Elem<DT>::T *o = z + (size_t)i * ZC;
    o[0] = Elem<DT>::make(v);
#pragma unroll
    for (int c = 1; c < ZC; ++c) o[c] = Elem<DT>::make(0.f);
}

// out[b][y][x] = 256 * (bias + sum over level-1 pixels (i, j) and taps (u, v)
// with f*i + u - 2 = y, f*j + v - 2 = x of T[b][i][j][5u + v]), rows i and
// columns j ascending.
__global__ void __launch_bounds__(256)
k_tv_final(const float *__restrict__ T, int B, int h, int w, int f, int H, int W,
           const float *__restrict__ bias, float *__restrict__ out) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int b = blockIdx.z;
    if (x >= W || y >= H) return;
    // i with 0 <= y + 2 - f i <= 4
    const int ilo = max(0, (y - 2 + f - 1 + 2 * f) / f - 2), ihi = min(h - 1, (y + 2) / f);
    const int jlo = max(0, (x - 2 + f - 1 + 2 * f) / f - 2), jhi = min(w - 1, (x + 2) / f);
    float s = 0.f;
    for (int i = ilo; i <= ihi; ++i) {
        const int u = y + 2 - f * i;
        for (int j = jlo; j <= jhi; ++j) {
            const int v = x + 2 - f * j;
            s += T[(((size_t)b * h + i) * w + j) * TC + u * TV_K + v];
        }
    }
    out[((size_t)b * H + y) * W + x] = 256.0f * (s + bias[0]);
}

__global__ void k_tv_copy(const float *__restrict__ src, int n, float *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

ConvSrc tsrc(const void *p, int C, int pitch, int coff, int hs, int ws, int kind, int sdt) {
    ConvSrc s{};
    s.ptr = p; s.kind = kind; s.C = C; s.pitch = pitch; s.coff = coff; s.hs = hs; s.ws = ws; s.sdt = sdt;
    return s;
}

// Form of the stride-2 deconvolutions: -1 by output size (polyphase from
// TV_PHASE_MIN_PIX output pixels: four launches beat one only when each has
// enough work), 0 always over the zero-inserted grid, 1 always polyphase.
std::atomic<int> g_tv_deconv_form{-1};
constexpr long long TV_PHASE_MIN_PIX = 131072;

bool tv_polyphase(int B, int Ho, int Wo) {
    const int f = g_tv_deconv_form.load();
    if (f >= 0) return f == 1;
    return (long long)B * Ho * Wo >= TV_PHASE_MIN_PIX;
}

// Feature extraction (FE_1 = conv5x5(X_0), FE_2 = conv5x5(X_1), 32 outputs
// each, leaky ReLU) as a direct stencil: with one input channel per branch an
// MFMA reduction would run almost empty.  A workgroup owns 16 x 4 coarse
// pixels; the X_0 / X_1 patch with its 2-pixel halo is built in LDS from the
// uint8 maps; wave g accumulates outputs 16g .. 16g + 15 (waves 0-1: FE_1 on
// X_0, 2-3: FE_2 on X_1) of every pixel in FP32 from weights staged once in
// LDS as FP32 [tap][output] (the packed layer: rows 0..31 on channel 0, rows
// 32..63 on channel 1), then stores them into channels 16..79 of the level-1
// map.
constexpr int FE_TW = 16, FE_TH = 4, FE_PW = FE_TW + 4, FE_PH = FE_TH + 4;

template <int DT>
__global__ void __launch_bounds__(256)
k_tv_fe(const uint8_t *__restrict__ disp, const uint8_t *__restrict__ img, int h, int w, float scale0,
        const typename Elem<DT>::T *__restrict__ wpk, int n_pad, int cin_pad, const float *__restrict__ bias,
        typename Elem<DT>::T *__restrict__ out) {
    __shared__ float xs[2][FE_PH * FE_PW];
    __shared__ __attribute__((aligned(16))) float wsh[TV_TAPS * 64];  // [tap][output], FP32
    const int b = blockIdx.z;
    const int x0 = blockIdx.x * FE_TW, y0 = blockIdx.y * FE_TH;
    const size_t ib = (size_t)b * h * w;
    for (int e = threadIdx.x; e < TV_TAPS * 64; e += 256) {
        const int t = e >> 6, o = e & 63;
        wsh[e] = Elem<DT>::load(wpk + ((size_t)t * n_pad + o) * cin_pad + (o >> 5));
    }
    for (int e = threadIdx.x; e < FE_PH * FE_PW; e += 256) {
        const int py = e / FE_PW, px = e - py * FE_PW;
        const int y = y0 + py - 2, x = x0 + px - 2;
        float a = 0.f, c = 0.f;
        if (y >= 0 && y < h && x >= 0 && x < w) {
            a = scale0 * (float)disp[ib + (size_t)y * w + x];
            c = (float)img[ib + (size_t)y * w + x] * (1.0f / 256.0f);
        }
        xs[0][e] = a;
        xs[1][e] = c;
    }
    __syncthreads();
    // the output group is the wave's: the weight reads below are the same LDS
    // address for the whole wave (a broadcast)
    const int lane = threadIdx.x & 63, grp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tx = lane & (FE_TW - 1), ty = lane / FE_TW;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= w || y >= h) return;
    const int ch = grp >> 1, o0 = grp * 16;
    const float *xp = xs[ch];
    float acc[16];
#pragma unroll
    for (int o = 0; o < 16; ++o) acc[o] = bias[o0 + o];
#pragma unroll
    for (int t = 0; t < TV_TAPS; ++t) {
        const int u = t / TV_K, v = t % TV_K;
        const float xv = xp[(ty + u) * FE_PW + tx + v];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const f32x4 wv = *(const f32x4 *)&wsh[t * 64 + o0 + 4 * q];
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[4 * q + i] = fmaf(wv[i], xv, acc[4 * q + i]);
        }
    }
    typename Elem<DT>::T *op = out + ((ib + (size_t)y * w + x) * L1C + 16 + o0);
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        const float r = acc[o] > 0.f ? acc[o] : 0.1f * acc[o];
        op[o] = Elem<DT>::make(r);
    }
}

sv_status tv_fe(const TvShape &s, const void *packed, const uint8_t *disp, const uint8_t *img, int B, int h, int w,
                int f, void *L1, const int *cfg, int only, hipStream_t st) {
    (void)cfg;
    if (only >= 0 && only != T_FE) return SV_OK;
    const dim3 grid(cdiv(w, FE_TW), cdiv(h, FE_TH), B);
    const float sc = (float)f / 256.0f;
    const float *bias = (const float *)((const char *)packed + s.b_off[T_FE]);
    const void *wp = (const char *)packed + s.w_off[T_FE];
    switch (s.dtype) {
    case SV_F32: hipLaunchKernelGGL(k_tv_fe<SV_F32>, grid, dim3(256), 0, st, disp, img, h, w, sc, (const float *)wp, s.n_pad[T_FE], s.cin_pad[T_FE], bias, (float *)L1); break;
    case SV_BF16: hipLaunchKernelGGL(k_tv_fe<SV_BF16>, grid, dim3(256), 0, st, disp, img, h, w, sc, (const uint16_t *)wp, s.n_pad[T_FE], s.cin_pad[T_FE], bias, (uint16_t *)L1); break;
    default: hipLaunchKernelGGL(k_tv_fe<SV_F16>, grid, dim3(256), 0, st, disp, img, h, w, sc, (const uint16_t *)wp, s.n_pad[T_FE], s.cin_pad[T_FE], bias, (uint16_t *)L1); break;
    }
    SV_LAUNCH_CHECK("k_tv_fe");
    return SV_OK;
}

// A stride-2 deconvolution (D_2 or D) as four 3x3 correlations over its
// input, one per output parity class, each writing its pixels of the
// interleaved Ho x Wo output.
sv_status tv_deconv2(const TvShape &s, const void *packed, int li, ConvSrc src, int B, int Hi, int Wi, int Ho,
                     int Wo, void *out, int out_pitch, int out_coff, const int *cfg, int only, hipStream_t st) {
    if (only >= 0 && only != li) return SV_OK;
    for (int ph = 0; ph < 4; ++ph) {
        const int py = ph >> 1, px = ph & 1;
        ConvParams p{};
        p.src[0] = src;
        p.B = B; p.Hi = Hi; p.Wi = Wi;
        p.Ho = (Ho - py + 1) / 2; p.Wo = (Wo - px + 1) / 2;
        if (p.Ho <= 0 || p.Wo <= 0) continue;
        p.ophase = 1 + ph; p.Ho_full = Ho; p.Wo_full = Wo;
        p.Cin = src.C;
        p.Cout = kLayers[li].cout;
        p.cin_pad = s.cin_pad[li];
        p.n_pad = s.n_pad[li];
        p.wpk = (const char *)packed + s.ph_off[li][ph];
        p.bias = (const float *)((const char *)packed + s.b_off[li]);
        p.out = out; p.out_pitch = out_pitch; p.out_coff = out_coff;
        p.act = 1;
        SV_TRY_STATUS(launch_conv(s.dtype, 3, 1, cfg[li] % conv_num_tiles(), p, st));
    }
    return SV_OK;
}

// One launched layer with configuration cfg[li]; with only >= 0 every other
// layer is skipped (the autotuner times one layer at a time).
sv_status tv_layer(const TvShape &s, const void *packed, int li, ConvSrc s0, ConvSrc s1, int B, int Hi,
                   int Wi, int Ho, int Wo, void *out, int out_pitch, int out_coff, int out_f32, int act,
                   float *part, size_t part_bytes, const int *cfg, int only, hipStream_t st) {
    if (only >= 0 && only != li) return SV_OK;
    ConvParams p{};
    p.part = part;
    p.part_bytes = part_bytes;
    p.src[0] = s0; p.src[1] = s1;
    p.B = B; p.Hi = Hi; p.Wi = Wi; p.Ho = Ho; p.Wo = Wo;
    p.Cin = s0.C + (s1.kind ? s1.C : 0);
    p.Cout = kLayers[li].cout;
    p.cin_pad = s.cin_pad[li];
    p.n_pad = s.n_pad[li];
    p.wpk = (const char *)packed + s.w_off[li];
    p.bias = li == T_YP ? nullptr : (const float *)((const char *)packed + s.b_off[li]);
    p.out = out; p.out_pitch = out_pitch; p.out_coff = out_coff;
    p.act = act; p.out_f32 = out_f32;
    const int dt = li == T_YP ? SV_F32 : s.dtype;
    return launch_conv(dt, kLayers[li].k, kLayers[li].stride, cfg[li], p, st);
}

sv_status tv_forward(const TvShape &s, int f, const void *packed, const uint8_t *disp, const uint8_t *img,
                     int B, int H, int W, const float *eps, float *out, float *ml_user, void *ws,
                     hipStream_t st, int only = -1, const int *cfg_in = nullptr) {
    // cfg_in (nullable): this call's configurations (the autotuner's candidates)
    int cfg[T_NL];
    if (cfg_in) {
        for (int i = 0; i < T_NL; ++i) cfg[i] = cfg_in[i];
    } else {
        tv_layer_cfgs(s.dtype, f, B, H, W, cfg);
    }
    const TvLevels lv = tv_levels(f, H, W);
    const TvAct a = tv_act(s.es, lv, B);
    char *w = (char *)ws;
    void *L1 = w + a.L1, *L2 = w + a.L2, *L3 = w + a.L3, *Z = w + a.Z;
    // mu / sigma stay in the workspace (the backward reads them there); the
    // caller's buffer gets a copy
    float *ML = (float *)(w + a.ML);
    float *T = (float *)(w + a.T);
    float *part = (float *)(w + a.part);
    const int h1 = lv.h[1], w1 = lv.w[1], h2 = lv.h[2], w2 = lv.w[2], h3 = lv.h[3], w3 = lv.w[3];
    const ConvSrc none{};
    ConvSrc x0{};
    x0.ptr = disp; x0.img = img; x0.kind = SRC_X0; x0.C = 2; x0.hs = h1; x0.ws = w1;
    x0.scale0 = (float)f / 256.0f;
    // feature extraction: [FE_1 | FE_2] into level 1, channels 16..79
    SV_TRY_STATUS(tv_fe(s, packed, disp, img, B, h1, w1, f, L1, cfg, only, st));
    // encoder
    SV_TRY_STATUS(tv_layer(s, packed, T_EN1, tsrc(L1, 64, L1C, 16, h1, w1, SRC_TENSOR, 0), none, B, h1, w1, h2, w2,
                           L2, L2C, 16, 0, 1, part, a.part_bytes, cfg, only, st));
    SV_TRY_STATUS(tv_layer(s, packed, T_EN1R, tsrc(L2, 16, L2C, 16, h2, w2, SRC_TENSOR, 0), none, B, h2, w2, h2, w2,
                           L2, L2C, 32, 0, 1, part, a.part_bytes, cfg, only, st));
    SV_TRY_STATUS(tv_layer(s, packed, T_EN2, tsrc(L2, 24, L2C, 16, h2, w2, SRC_TENSOR, 0), none, B, h2, w2, h3, w3,
                           L3, L3C, 32, 0, 1, part, a.part_bytes, cfg, only, st));
    SV_TRY_STATUS(tv_layer(s, packed, T_EN2R, tsrc(L3, 32, L3C, 32, h3, w3, SRC_TENSOR, 0), none, B, h3, w3, h3, w3,
                           L3, L3C, 64, 0, 1, part, a.part_bytes, cfg, only, st));
    // mu & sigma (FP32), then Eq. (8)
    SV_TRY_STATUS(tv_layer(s, packed, T_MS, tsrc(L3, 48, L3C, 32, h3, w3, SRC_TENSOR, 0), none, B, h3, w3, h3, w3,
                           ML, 2, 0, 1, 0, part, a.part_bytes, cfg, only, st));
    const int nl = B * h3 * w3;
    if (ml_user && only < 0) {
        hipLaunchKernelGGL(k_tv_copy, dim3(cdiv(2 * nl, 256)), dim3(256), 0, st, ML, 2 * nl, ml_user);
        SV_LAUNCH_CHECK("k_tv_copy");
    }
    if (only < 0) switch (s.dtype) {
    case SV_F32: hipLaunchKernelGGL(k_tv_reparam<SV_F32>, dim3(cdiv(nl, 256)), dim3(256), 0, st, ML, eps, nl, (float *)Z); break;
    case SV_BF16: hipLaunchKernelGGL(k_tv_reparam<SV_BF16>, dim3(cdiv(nl, 256)), dim3(256), 0, st, ML, eps, nl, (uint16_t *)Z); break;
    default: hipLaunchKernelGGL(k_tv_reparam<SV_F16>, dim3(cdiv(nl, 256)), dim3(256), 0, st, ML, eps, nl, (uint16_t *)Z); break;
    }
    SV_LAUNCH_CHECK("k_tv_reparam");
    // decoder
    SV_TRY_STATUS(tv_layer(s, packed, T_D1, tsrc(Z, 1, ZC, 0, h3, w3, SRC_TENSOR, 0), none, B, h3, w3, h3, w3,
                           L3, L3C, 0, 0, 1, part, a.part_bytes, cfg, only, st));
    SV_TRY_STATUS(tv_layer(s, packed, T_D1R, tsrc(L3, 80, L3C, 0, h3, w3, SRC_TENSOR, 0), none, B, h3, w3, h3, w3,
                           L3, L3C, 80, 0, 1, part, a.part_bytes, cfg, only, st));
    // stride-2 deconvolutions: polyphase for large outputs, else one launch over
    // the zero-inserted grid (2n - 1 samples per axis)
    if (tv_polyphase(B, h2, w2))
        SV_TRY_STATUS(tv_deconv2(s, packed, T_D2, tsrc(L3, 96, L3C, 0, h3, w3, SRC_TENSOR, 0), B, h3, w3, h2, w2,
                                 L2, L2C, 0, cfg, only, st));
    else
        SV_TRY_STATUS(tv_layer(s, packed, T_D2, tsrc(L3, 96, L3C, 0, h3, w3, SRC_ZINS, 0), none, B, 2 * h3 - 1,
                               2 * w3 - 1, h2, w2, L2, L2C, 0, 0, 1, part, a.part_bytes, cfg, only, st));
    SV_TRY_STATUS(tv_layer(s, packed, T_D2R, tsrc(L2, 40, L2C, 0, h2, w2, SRC_TENSOR, 0), none, B, h2, w2, h2, w2,
                           L2, L2C, 40, 0, 1, part, a.part_bytes, cfg, only, st));
    if (tv_polyphase(B, h1, w1))
        SV_TRY_STATUS(tv_deconv2(s, packed, T_D, tsrc(L2, 48, L2C, 0, h2, w2, SRC_TENSOR, 0), B, h2, w2, h1, w1,
                                 L1, L1C, 0, cfg, only, st));
    else
        SV_TRY_STATUS(tv_layer(s, packed, T_D, tsrc(L2, 48, L2C, 0, h2, w2, SRC_ZINS, 0), none, B, 2 * h2 - 1,
                               2 * w2 - 1, h1, w1, L1, L1C, 0, 0, 1, part, a.part_bytes, cfg, only, st));
    // upsampling layer: tap projection of [D | FE_1 | FE_2 | X_0 X_1] (FP32
    // weights; the map is read in its stored dtype), then the gather
    const int sdt = s.dtype == SV_F32 ? 0 : 1 + s.dtype;
    SV_TRY_STATUS(tv_layer(s, packed, T_YP, tsrc(L1, 80, L1C, 0, h1, w1, SRC_TENSOR, sdt), x0, B, h1, w1, h1, w1,
                           T, TC, 0, 1, 0, part, a.part_bytes, cfg, only, st));
    if (only >= 0) return SV_OK;
    hipLaunchKernelGGL(k_tv_final, dim3(cdiv(W, 64), cdiv(H, 4), B), dim3(256), 0, st, T, B, h1, w1, f, H, W,
                       (const float *)((const char *)packed + s.b_off[T_YP]), out);
    SV_LAUNCH_CHECK("k_tv_final");
    return SV_OK;
}

// ---- backward ----------------------------------------------------------------------
// Gradient maps (FP32 NHWC): one per level, channel ranges as in the forward
// maps; dZ [px3]; d(mu, sigma) [px3][8] (channels 2..7 zero, so that the 1x1
// input-gradient convolution reads whole channel groups); the tap gradients
// of the upsampling layer [px1][32] (taps 25..31 zero).
constexpr int DMLC = 8;
struct TvBwd { size_t dL1, dL2, dL3, dZ, dML, dT, part, sum, total; };

TvBwd tv_bwd_layout(const TvShape &s, const TvLevels &lv, int B) {
    auto px = [&](int k) { return (size_t)B * lv.h[k] * lv.w[k]; };
    TvBwd l{};
    size_t o = 0;
    auto take = [&](size_t floats) { size_t r = o; o = align256(o + floats * sizeof(float)); return r; };
    l.dL1 = take(px(1) * L1C);
    l.dL2 = take(px(2) * L2C);
    l.dL3 = take(px(3) * L3C);
    l.dZ = take(px(3));
    l.dML = take(px(3) * DMLC);
    l.dT = take(px(1) * TC);
    // weight-gradient partial sums of the largest layer (layers run one after another)
    size_t mx = 0;
    for (int i = 0; i < T_NL; ++i) {
        const int k = kOutLevel[i];
        mx = std::max(mx, wgrad_partial_floats(B, lv.h[k], lv.w[k], kLayers[i].cin, kLayers[i].cout, kLayers[i].k));
    }
    l.part = take(mx);
    l.sum = take(256 + 1);
    l.total = o;
    (void)s;
    return l;
}

// dT[b][i][j][t] = 256 * dout[b][f i + u - 2][f j + v - 2] (t = 5u + v; 0 where
// that pixel is outside the image, and for t >= 25): each tap of a coarse
// pixel lands on exactly one full-resolution pixel.
__global__ void k_tv_final_bwd(const float *__restrict__ dout, int B, int h, int w, int f, int H, int W,
                               float *__restrict__ dT) {
    const size_t n = (size_t)B * h * w * TC;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int t = (int)(e % TC);
        const size_t pix = e / TC;
        const int j = (int)(pix % w), i = (int)((pix / w) % h), b = (int)(pix / ((size_t)w * h));
        float v = 0.f;
        if (t < TV_TAPS) {
            const int y = f * i + t / TV_K - 2, x = f * j + t % TV_K - 2;
            if (y >= 0 && y < H && x >= 0 && x < W) v = 256.0f * dout[((size_t)b * H + y) * W + x];
        }
        dT[e] = v;
    }
}

// sum of 256 * dout (Y's bias), two fixed-order passes
__global__ void __launch_bounds__(256) k_tv_sum_partial(const float *__restrict__ x, int64_t n, float *__restrict__ part) {
    __shared__ double sh[256];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) acc += (double)x[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = (float)sh[0];
}

__global__ void __launch_bounds__(256) k_tv_sum_final(const float *__restrict__ part, float scale, float *__restrict__ out) {
    __shared__ double sh[256];
    sh[threadIdx.x] = (double)part[threadIdx.x];
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)(scale * sh[0]);
}

// leaky-ReLU derivative from the stored output (0.1 where it is <= 0)
template <int DT>
__global__ void k_tv_mask(float *__restrict__ g, int gpitch, int gcoff, const typename Elem<DT>::T *__restrict__ act,
                          int apitch, int acoff, int C, size_t npix) {
    const size_t n = npix * C;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t pix = e / C;
        const int c = (int)(e - pix * C);
        const float a = Elem<DT>::load(act + pix * apitch + acoff + c);
        if (!(a > 0.f)) g[pix * gpitch + gcoff + c] *= 0.1f;
    }
}

// Eq. (8) backward: d mu = dz (+ the loss's), d sigma = dz * eps * exp(sigma - 1) (+ the loss's)
__global__ void k_tv_reparam_bwd(const float *__restrict__ dz, const float *__restrict__ ml, const float *__restrict__ eps,
                                 const float *__restrict__ dms, int n, float *__restrict__ dml) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float dm = dz[i], ds = eps ? dz[i] * eps[i] * expf(ml[2 * i + 1] - 1.0f) : 0.f;
    if (dms) { dm += dms[2 * i]; ds += dms[2 * i + 1]; }
    float *o = dml + (size_t)i * DMLC;
    o[0] = dm;
    o[1] = ds;
#pragma unroll
    for (int c = 2; c < DMLC; ++c) o[c] = 0.f;
}

// Canonical weight and bias gradient of one canonical layer from the partial
// sums of the launched layer's weight gradient: row = row0 + o (proj: the
// tap), tap = the canonical tap (flipped for a deconvolution's stride-1 form),
// column = cmap[canonical input channel].
struct GradJob {
    int cout, cin, k, row0, flip, proj, bias;
    int splits, o_pad, taps, cinp;
    int cmap[96];
};

__global__ void k_tv_grad_reduce(const GradJob j, const float *__restrict__ part, float *__restrict__ grad) {
    const int kk = j.k * j.k;
    const int nw = j.cout * j.cin * kk;
    const int n = nw + (j.bias ? j.cout : 0);
    const float *part_b = part + (size_t)j.splits * j.o_pad * j.taps * j.cinp;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        float acc = 0.f;
        if (e < nw) {
            const int o = e / (j.cin * kk), ci = (e / kk) % j.cin, t = e % kk;
            const int col = j.cmap[ci];
            const int row = j.proj ? t : j.row0 + o;
            const int tap = j.proj ? 0 : (j.flip ? kk - 1 - t : t);
            if (col >= 0)
                for (int sp = 0; sp < j.splits; ++sp)
                    acc += part[(((size_t)sp * j.o_pad + row) * j.taps + tap) * j.cinp + col];
        } else {
            const int o = e - nw;
            for (int sp = 0; sp < j.splits; ++sp) acc += part_b[(size_t)sp * j.o_pad + j.row0 + o];
        }
        grad[e] = acc;
    }
}

ConvSrc fsrc(const float *p, int C, int pitch, int coff, int hs, int ws, int kind) {
    return tsrc(p, C, pitch, coff, hs, ws, kind, SDT_F32);
}

// Input gradient of launched layer li through the forward convolution kernel
// and the adjoint pack: `dy` is the output gradient as a source (plain, or
// zero-inserted for a stride-2 convolution); out / add give the target range.
sv_status tv_dgrad(const TvShape &s, const void *packed, int li, ConvSrc dy, int stride, int B, int Hi, int Wi,
                   int Ho, int Wo, float *out, int out_pitch, int out_coff, bool add, hipStream_t st) {
    ConvParams p{};
    p.src[0] = dy;
    p.B = B; p.Hi = Hi; p.Wi = Wi; p.Ho = Ho; p.Wo = Wo;
    p.Cin = dy.C;
    p.Cout = kAdjRows[li];
    p.cin_pad = s.bcin_pad[li];
    p.n_pad = s.bn_pad[li];
    p.wpk = (const char *)packed + s.bw_off[li];
    p.out = out; p.out_pitch = out_pitch; p.out_coff = out_coff; p.out_f32 = 1;
    if (add) { p.add = out; p.add_pitch = out_pitch; p.add_coff = out_coff; }
    const int cfg = p.Cout <= 16 ? 5 : 2;
    return launch_conv(li == T_YP ? SV_F32 : s.dtype, kLayers[li].k, stride, cfg, p, st);
}

sv_status tv_backward(const TvShape &s, int f, const void *packed, const uint8_t *disp, const uint8_t *img, int B,
                      int H, int W, const float *eps, const void *fws, const float *dout, const float *dms,
                      float *grad, void *ws, hipStream_t st) {
    const TvLevels lv = tv_levels(f, H, W);
    const TvAct a = tv_act(s.es, lv, B);
    const TvBwd l = tv_bwd_layout(s, lv, B);
    const char *fw = (const char *)fws;
    const void *L1 = fw + a.L1, *L2 = fw + a.L2, *L3 = fw + a.L3, *Z = fw + a.Z;
    const float *ML = (const float *)(fw + a.ML);
    char *bw = (char *)ws;
    float *dL1 = (float *)(bw + l.dL1), *dL2 = (float *)(bw + l.dL2), *dL3 = (float *)(bw + l.dL3);
    float *dZ = (float *)(bw + l.dZ), *dML = (float *)(bw + l.dML), *dT = (float *)(bw + l.dT);
    float *part = (float *)(bw + l.part), *sum = (float *)(bw + l.sum);
    const int h1 = lv.h[1], w1 = lv.w[1], h2 = lv.h[2], w2 = lv.w[2], h3 = lv.h[3], w3 = lv.w[3];
    const size_t p1 = (size_t)B * h1 * w1, p2 = (size_t)B * h2 * w2, p3 = (size_t)B * h3 * w3;
    const int sdt = s.dtype == SV_F32 ? 0 : 1 + s.dtype;  // the maps' storage, seen from an FP32 launch
    const ConvSrc none{};
    ConvSrc x0{};
    x0.ptr = disp; x0.img = img; x0.kind = SRC_X0; x0.C = 2; x0.hs = h1; x0.ws = w1;
    x0.scale0 = (float)f / 256.0f;
    auto blocks = [](size_t n) { return (unsigned)std::min<size_t>((n + 255) / 256, 4096); };

    // weight gradient of launched layer li into the canonical slices of `jobs`
    auto wgrad = [&](int li, int ks, int stride, ConvSrc s0, ConvSrc s1, int Hi, int Wi, int Ho, int Wo,
                     const float *dy, int dy_pitch, std::initializer_list<GradJob> jobs,
                     std::initializer_list<int> canons) -> sv_status {
        WgradShape sh{};
        SV_TRY_STATUS(launch_wgrad_partials(li == T_YP ? SV_F32 : s.dtype, ks, stride, s0, s1, B, Hi, Wi, Ho, Wo,
                                            kLayers[li].cout, dy, dy_pitch, part, sh, st));
        auto cit = canons.begin();
        for (GradJob j : jobs) {
            j.splits = sh.splits; j.o_pad = sh.o_pad; j.taps = sh.taps; j.cinp = sh.cinp;
            const int n = j.cout * j.cin * j.k * j.k + (j.bias ? j.cout : 0);
            hipLaunchKernelGGL(k_tv_grad_reduce, dim3(cdiv(n, 256)), dim3(256), 0, st, j, part, grad + canon_off(*cit));
            SV_LAUNCH_CHECK("k_tv_grad_reduce");
            ++cit;
        }
        return SV_OK;
    };
    auto job = [&](int canon, int row0, bool flip, auto colmap) {
        GradJob j{};
        j.cout = kCanon[canon].cout; j.cin = kCanon[canon].cin; j.k = kCanon[canon].k;
        j.row0 = row0; j.flip = flip; j.proj = canon == C_Y; j.bias = canon != C_Y;
        for (int q = 0; q < 96; ++q) j.cmap[q] = q < j.cin ? colmap(q) : -1;
        return j;
    };
    auto idc = [](int q) { return q; };
    auto mask = [&](float *g, int gpitch, int gcoff, const void *act, int apitch, int acoff, int C, size_t npix) -> sv_status {
        switch (s.dtype) {
        case SV_F32: hipLaunchKernelGGL(k_tv_mask<SV_F32>, dim3(blocks(npix * C)), dim3(256), 0, st, g, gpitch, gcoff, (const float *)act, apitch, acoff, C, npix); break;
        case SV_BF16: hipLaunchKernelGGL(k_tv_mask<SV_BF16>, dim3(blocks(npix * C)), dim3(256), 0, st, g, gpitch, gcoff, (const uint16_t *)act, apitch, acoff, C, npix); break;
        default: hipLaunchKernelGGL(k_tv_mask<SV_F16>, dim3(blocks(npix * C)), dim3(256), 0, st, g, gpitch, gcoff, (const uint16_t *)act, apitch, acoff, C, npix); break;
        }
        SV_LAUNCH_CHECK("k_tv_mask");
        return SV_OK;
    };

    // upsampling layer: tap gradients, Y's bias, its projection's weights and input gradient
    hipLaunchKernelGGL(k_tv_final_bwd, dim3(blocks(p1 * TC)), dim3(256), 0, st, dout, B, h1, w1, f, H, W, dT);
    SV_LAUNCH_CHECK("k_tv_final_bwd");
    hipLaunchKernelGGL(k_tv_sum_partial, dim3(256), dim3(256), 0, st, dout, (int64_t)B * H * W, sum);
    hipLaunchKernelGGL(k_tv_sum_final, dim3(1), dim3(256), 0, st, sum, 256.0f, grad + canon_off(C_Y) + 81 * 25);
    SV_LAUNCH_CHECK("k_tv_sum");
    SV_TRY_STATUS(wgrad(T_YP, 1, 1, tsrc(L1, 80, L1C, 0, h1, w1, SRC_TENSOR, sdt), x0, h1, w1, h1, w1, dT, TC,
                        {job(C_Y, 0, false, [](int q) { return q < 16 ? q : (q == 16 ? 80 : q - 1); })}, {C_Y}));
    SV_TRY_STATUS(tv_dgrad(s, packed, T_YP, fsrc(dT, TV_TAPS, TC, 0, h1, w1, SRC_TENSOR), 1, B, h1, w1, h1, w1,
                           dL1, L1C, 0, false, st));
    // D (deconvolution into level 1)
    SV_TRY_STATUS(mask(dL1, L1C, 0, L1, L1C, 0, 16, p1));
    SV_TRY_STATUS(wgrad(T_D, 5, 1, tsrc(L2, 48, L2C, 0, h2, w2, SRC_ZINS, 0), none, 2 * h2 - 1, 2 * w2 - 1, h1, w1,
                        dL1, L1C, {job(C_D, 0, true, idc)}, {C_D}));
    SV_TRY_STATUS(tv_dgrad(s, packed, T_D, fsrc(dL1, 16, L1C, 0, h1, w1, SRC_TENSOR), 2, B, h1, w1, h2, w2,
                           dL2, L2C, 0, false, st));
    // D_2_R
    SV_TRY_STATUS(mask(dL2, L2C, 40, L2, L2C, 40, 8, p2));
    SV_TRY_STATUS(wgrad(T_D2R, 5, 1, tsrc(L2, 40, L2C, 0, h2, w2, SRC_TENSOR, 0), none, h2, w2, h2, w2, dL2 + 40, L2C,
                        {job(C_D2R, 0, false, idc)}, {C_D2R}));
    SV_TRY_STATUS(tv_dgrad(s, packed, T_D2R, fsrc(dL2, 8, L2C, 40, h2, w2, SRC_TENSOR), 1, B, h2, w2, h2, w2,
                           dL2, L2C, 0, true, st));
    // D_2 (deconvolution into level 2)
    SV_TRY_STATUS(mask(dL2, L2C, 0, L2, L2C, 0, 16, p2));
    SV_TRY_STATUS(wgrad(T_D2, 5, 1, tsrc(L3, 96, L3C, 0, h3, w3, SRC_ZINS, 0), none, 2 * h3 - 1, 2 * w3 - 1, h2, w2,
                        dL2, L2C, {job(C_D2, 0, true, idc)}, {C_D2}));
    SV_TRY_STATUS(tv_dgrad(s, packed, T_D2, fsrc(dL2, 16, L2C, 0, h2, w2, SRC_TENSOR), 2, B, h2, w2, h3, w3,
                           dL3, L3C, 0, false, st));
    // D_1_R
    SV_TRY_STATUS(mask(dL3, L3C, 80, L3, L3C, 80, 16, p3));
    SV_TRY_STATUS(wgrad(T_D1R, 5, 1, tsrc(L3, 80, L3C, 0, h3, w3, SRC_TENSOR, 0), none, h3, w3, h3, w3, dL3 + 80, L3C,
                        {job(C_D1R, 0, false, idc)}, {C_D1R}));
    SV_TRY_STATUS(tv_dgrad(s, packed, T_D1R, fsrc(dL3, 16, L3C, 80, h3, w3, SRC_TENSOR), 1, B, h3, w3, h3, w3,
                           dL3, L3C, 0, true, st));
    // D_1 (1x1 deconvolution of z)
    SV_TRY_STATUS(mask(dL3, L3C, 0, L3, L3C, 0, 32, p3));
    SV_TRY_STATUS(wgrad(T_D1, 1, 1, tsrc(Z, 1, ZC, 0, h3, w3, SRC_TENSOR, 0), none, h3, w3, h3, w3, dL3, L3C,
                        {job(C_D1, 0, false, idc)}, {C_D1}));
    SV_TRY_STATUS(tv_dgrad(s, packed, T_D1, fsrc(dL3, 32, L3C, 0, h3, w3, SRC_TENSOR), 1, B, h3, w3, h3, w3,
                           dZ, 1, 0, false, st));
    // Eq. (8), then the head
    hipLaunchKernelGGL(k_tv_reparam_bwd, dim3(cdiv((int)p3, 256)), dim3(256), 0, st, dZ, ML, eps, dms, (int)p3, dML);
    SV_LAUNCH_CHECK("k_tv_reparam_bwd");
    SV_TRY_STATUS(wgrad(T_MS, 1, 1, tsrc(L3, 48, L3C, 32, h3, w3, SRC_TENSOR, 0), none, h3, w3, h3, w3, dML, DMLC,
                        {job(C_MS, 0, false, idc)}, {C_MS}));
    SV_TRY_STATUS(tv_dgrad(s, packed, T_MS, fsrc(dML, 2, DMLC, 0, h3, w3, SRC_TENSOR), 1, B, h3, w3, h3, w3,
                           dL3, L3C, 32, true, st));
    // EN_2_R
    SV_TRY_STATUS(mask(dL3, L3C, 64, L3, L3C, 64, 16, p3));
    SV_TRY_STATUS(wgrad(T_EN2R, 5, 1, tsrc(L3, 32, L3C, 32, h3, w3, SRC_TENSOR, 0), none, h3, w3, h3, w3, dL3 + 64, L3C,
                        {job(C_EN2R, 0, false, idc)}, {C_EN2R}));
    SV_TRY_STATUS(tv_dgrad(s, packed, T_EN2R, fsrc(dL3, 16, L3C, 64, h3, w3, SRC_TENSOR), 1, B, h3, w3, h3, w3,
                           dL3, L3C, 32, true, st));
    // EN_2 (stride 2: its input gradient runs over the zero-inserted output gradient)
    SV_TRY_STATUS(mask(dL3, L3C, 32, L3, L3C, 32, 32, p3));
    SV_TRY_STATUS(wgrad(T_EN2, 5, 2, tsrc(L2, 24, L2C, 16, h2, w2, SRC_TENSOR, 0), none, h2, w2, h3, w3, dL3 + 32, L3C,
                        {job(C_EN2, 0, false, idc)}, {C_EN2}));
    SV_TRY_STATUS(tv_dgrad(s, packed, T_EN2, fsrc(dL3, 32, L3C, 32, h3, w3, SRC_ZINS), 1, B, 2 * h3 - 1, 2 * w3 - 1,
                           h2, w2, dL2, L2C, 16, true, st));
    // EN_1_R
    SV_TRY_STATUS(mask(dL2, L2C, 32, L2, L2C, 32, 8, p2));
    SV_TRY_STATUS(wgrad(T_EN1R, 5, 1, tsrc(L2, 16, L2C, 16, h2, w2, SRC_TENSOR, 0), none, h2, w2, h2, w2, dL2 + 32, L2C,
                        {job(C_EN1R, 0, false, idc)}, {C_EN1R}));
    SV_TRY_STATUS(tv_dgrad(s, packed, T_EN1R, fsrc(dL2, 8, L2C, 32, h2, w2, SRC_TENSOR), 1, B, h2, w2, h2, w2,
                           dL2, L2C, 16, true, st));
    // EN_1
    SV_TRY_STATUS(mask(dL2, L2C, 16, L2, L2C, 16, 16, p2));
    SV_TRY_STATUS(wgrad(T_EN1, 5, 2, tsrc(L1, 64, L1C, 16, h1, w1, SRC_TENSOR, 0), none, h1, w1, h2, w2, dL2 + 16, L2C,
                        {job(C_EN1, 0, false, idc)}, {C_EN1}));
    SV_TRY_STATUS(tv_dgrad(s, packed, T_EN1, fsrc(dL2, 16, L2C, 16, h2, w2, SRC_ZINS), 1, B, 2 * h2 - 1, 2 * w2 - 1,
                           h1, w1, dL1, L1C, 16, true, st));
    // FE_1 (rows 0..31, input channel 0) and FE_2 (rows 32..63, channel 1)
    SV_TRY_STATUS(mask(dL1, L1C, 16, L1, L1C, 16, 64, p1));
    SV_TRY_STATUS(wgrad(T_FE, 5, 1, x0, none, h1, w1, h1, w1, dL1 + 16, L1C,
                        {job(C_FE1, 0, false, [](int) { return 0; }), job(C_FE2, 32, false, [](int) { return 1; })},
                        {C_FE1, C_FE2}));
    return SV_OK;
}

// ---- loss (Eqs. (9)-(11)) -----------------------------------------------------------
constexpr int TL_BLOCKS = 256, TL_THREADS = 256;

__device__ __forceinline__ double tl_block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int k = TL_THREADS / 2; k > 0; k >>= 1) {
        if (t < k) sh[t] += sh[t + k];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// per block: sum |out - gt| (noc + occ), the occ count and the KL sum
__global__ void __launch_bounds__(TL_THREADS)
k_tv_loss_partial(const float *__restrict__ out, const float *__restrict__ gt, const uint8_t *__restrict__ noc,
                  const uint8_t *__restrict__ occ, int64_t n, const float *__restrict__ ml, int64_t nl,
                  double *__restrict__ part) {
    __shared__ double sh[TL_THREADS];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    double s = 0.0, cnt = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += TL_THREADS) {
        const double a = fabs((double)out[i] - (double)gt[i]);
        const int m = (noc[i] ? 1 : 0) + (occ[i] ? 1 : 0);
        s += a * m;
        cnt += occ[i] ? 1.0 : 0.0;
    }
    const int64_t perl = (nl + gridDim.x - 1) / gridDim.x;
    const int64_t llo = blockIdx.x * perl, lhi = llo + perl < nl ? llo + perl : nl;
    double k = 0.0;
    for (int64_t i = llo + threadIdx.x; i < lhi; i += TL_THREADS) {
        const double m = (double)ml[2 * i] - 1.0, sg = (double)ml[2 * i + 1] - 1.0;
        k += 0.5 * (m * m - 1.0 + exp(2.0 * sg) - 2.0 * sg);
    }
    s = tl_block_sum(s, sh);
    cnt = tl_block_sum(cnt, sh);
    k = tl_block_sum(k, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = s;
        part[3 * blockIdx.x + 1] = cnt;
        part[3 * blockIdx.x + 2] = k;
    }
}

// loss_out = [total, 256 * Loss_1, 256 * Loss_2]; part[3 * TL_BLOCKS] keeps the
// ground-truth count for the gradient kernel
__global__ void __launch_bounds__(TL_THREADS)
k_tv_loss_final(double *__restrict__ part, int64_t nl, float *__restrict__ loss_out) {
    __shared__ double sh[TL_THREADS];
    double s = 0.0, c = 0.0, k = 0.0;
    for (int i = threadIdx.x; i < TL_BLOCKS; i += TL_THREADS) {
        s += part[3 * i];
        c += part[3 * i + 1];
        k += part[3 * i + 2];
    }
    s = tl_block_sum(s, sh);
    c = tl_block_sum(c, sh);
    k = tl_block_sum(k, sh);
    if (threadIdx.x == 0) {
        const double nn = c > 1.0 ? c : 1.0;
        const double l1 = s / nn, l2 = nl > 0 ? 256.0 * k / (double)nl : 0.0;
        loss_out[0] = (float)(l1 + l2);
        loss_out[1] = (float)l1;
        loss_out[2] = (float)l2;
        part[3 * TL_BLOCKS] = nn;
    }
}

__global__ void k_tv_loss_grad(const float *__restrict__ out, const float *__restrict__ gt,
                               const uint8_t *__restrict__ noc, const uint8_t *__restrict__ occ, int64_t n,
                               const float *__restrict__ ml, int64_t nl, const double *__restrict__ part,
                               float *__restrict__ dout, float *__restrict__ dml) {
    const double inv = 1.0 / part[3 * TL_BLOCKS];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (!dout) break;
        const float e = out[i] - gt[i];
        const int sg = (e > 0.f) - (e < 0.f);
        const int m = (noc[i] ? 1 : 0) + (occ[i] ? 1 : 0);
        dout[i] = (float)((double)(sg * m) * inv);
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nl; i += (int64_t)gridDim.x * blockDim.x) {
        if (!dml) break;
        const double m = (double)ml[2 * i] - 1.0, sgm = (double)ml[2 * i + 1] - 1.0;
        dml[2 * i] = (float)(256.0 * m / (double)nl);
        dml[2 * i + 1] = (float)(256.0 * (exp(2.0 * sgm) - 1.0) / (double)nl);
    }
}

}  // namespace

}  // namespace sv

using namespace sv;

extern "C" {

int64_t sv_tvae_param_count(void) { return canon_off(NCANON); }

size_t sv_tvae_packed_bytes(int dtype) {
    if (dtype != SV_F32 && dtype != SV_BF16 && dtype != SV_F16) return 0;
    return tv_shape(dtype).bytes;
}

sv_status sv_tvae_pack_weights(int dtype, const float *params, void *packed_out, void *stream) {
    if (!params || !packed_out) return SV_ERR_NULL;
    if (dtype != SV_F32 && dtype != SV_BF16 && dtype != SV_F16) return SV_ERR_DTYPE;
    if ((uintptr_t)packed_out % 256) return SV_ERR_RANGE;
    return tv_pack(tv_shape(dtype), params, packed_out, (hipStream_t)stream);
}

static bool tv_shape_ok(int factor, int B, int H, int W) {
    if (factor < 1 || factor > 8 || B < 1 || H < 1 || W < 1) return false;
    if ((int64_t)B * H * W >= ((int64_t)1 << 31)) return false;
    // one workgroup row per 4 images in z for the widest layer
    return (int64_t)B * 4 <= 65535;
}

size_t sv_tvae_workspace_bytes(int dtype, int factor, int B, int H, int W) {
    if (dtype != SV_F32 && dtype != SV_BF16 && dtype != SV_F16) return 0;
    if (!tv_shape_ok(factor, B, H, W)) return 0;
    return tv_act(dtype_bytes(dtype), tv_levels(factor, H, W), B).total;
}

sv_status sv_tvae_forward(int dtype, int factor, const void *packed_w, const uint8_t *disp_low,
                          const uint8_t *img_low, int B, int H, int W, const float *eps, float *out,
                          float *mu_sigma, void *workspace, size_t ws_bytes, void *stream) {
    if (!packed_w || !disp_low || !img_low || !out || !workspace) return SV_ERR_NULL;
    if (dtype != SV_F32 && dtype != SV_BF16 && dtype != SV_F16) return SV_ERR_DTYPE;
    if (factor < 1 || factor > 8) return SV_ERR_RANGE;
    if (!tv_shape_ok(factor, B, H, W)) return SV_ERR_SHAPE;
    if (ws_bytes < sv_tvae_workspace_bytes(dtype, factor, B, H, W)) return SV_ERR_WORKSPACE;
    if ((uintptr_t)workspace % 256 || (uintptr_t)packed_w % 256) return SV_ERR_RANGE;
    return tv_forward(tv_shape(dtype), factor, packed_w, disp_low, img_low, B, H, W, eps, out, mu_sigma,
                      workspace, (hipStream_t)stream);
}

size_t sv_tvae_loss_workspace_bytes(void) { return sizeof(double) * (3 * TL_BLOCKS + 1); }

sv_status sv_tvae_loss(const float *out, const float *gt, const uint8_t *noc, const uint8_t *occ, int64_t n,
                       const float *mu_sigma, int64_t n_lat, float *loss_out, float *dout, float *dmu_sigma,
                       void *workspace, size_t ws_bytes, void *stream) {
    if (!out || !gt || !noc || !occ || !mu_sigma || !loss_out || !workspace) return SV_ERR_NULL;
    if (n <= 0 || n_lat <= 0) return SV_ERR_SHAPE;
    if (ws_bytes < sv_tvae_loss_workspace_bytes()) return SV_ERR_WORKSPACE;
    if ((uintptr_t)workspace % 8) return SV_ERR_RANGE;
    hipStream_t st = (hipStream_t)stream;
    double *part = (double *)workspace;
    hipLaunchKernelGGL(k_tv_loss_partial, dim3(TL_BLOCKS), dim3(TL_THREADS), 0, st, out, gt, noc, occ, n, mu_sigma,
                       n_lat, part);
    SV_LAUNCH_CHECK("k_tv_loss_partial");
    hipLaunchKernelGGL(k_tv_loss_final, dim3(1), dim3(TL_THREADS), 0, st, part, n_lat, loss_out);
    SV_LAUNCH_CHECK("k_tv_loss_final");
    if (dout || dmu_sigma) {
        const int64_t m = n > n_lat ? n : n_lat;
        const int blocks = (int)std::min<int64_t>((m + 255) / 256, 4096);
        hipLaunchKernelGGL(k_tv_loss_grad, dim3(blocks), dim3(256), 0, st, out, gt, noc, occ, n, mu_sigma, n_lat,
                           (const double *)part, dout, dmu_sigma);
        SV_LAUNCH_CHECK("k_tv_loss_grad");
    }
    return SV_OK;
}

sv_status sv_tvae_set_layer_cfg(int layer, int cfg) {
    if (layer < 0 || layer >= T_NL) return SV_ERR_RANGE;
    if (cfg < -1 || cfg >= conv_num_cfgs()) return SV_ERR_RANGE;
    g_tv_cfg[layer].store(cfg);
    return SV_OK;
}

int sv_tvae_num_layers(void) { return T_NL; }

sv_status sv_tvae_set_deconv_form(int form) {
    if (form < -1 || form > 1) return SV_ERR_RANGE;
    g_tv_deconv_form.store(form);
    return SV_OK;
}

size_t sv_tvae_backward_workspace_bytes(int dtype, int factor, int B, int H, int W) {
    if (dtype != SV_F32 && dtype != SV_BF16 && dtype != SV_F16) return 0;
    if (!tv_shape_ok(factor, B, H, W)) return 0;
    return tv_bwd_layout(tv_shape(dtype), tv_levels(factor, H, W), B).total;
}

sv_status sv_tvae_backward(int dtype, int factor, const void *packed_w, const uint8_t *disp_low,
                           const uint8_t *img_low, int B, int H, int W, const float *eps,
                           const void *fwd_workspace, const float *dout, const float *dmu_sigma, float *grad_out,
                           void *workspace, size_t ws_bytes, void *stream) {
    if (!packed_w || !disp_low || !img_low || !fwd_workspace || !dout || !grad_out || !workspace) return SV_ERR_NULL;
    if (dtype != SV_F32 && dtype != SV_BF16 && dtype != SV_F16) return SV_ERR_DTYPE;
    if (factor < 1 || factor > 8) return SV_ERR_RANGE;
    if (!tv_shape_ok(factor, B, H, W)) return SV_ERR_SHAPE;
    if (ws_bytes < sv_tvae_backward_workspace_bytes(dtype, factor, B, H, W)) return SV_ERR_WORKSPACE;
    if ((uintptr_t)workspace % 256 || (uintptr_t)fwd_workspace % 256 || (uintptr_t)packed_w % 256) return SV_ERR_RANGE;
    return tv_backward(tv_shape(dtype), factor, packed_w, disp_low, img_low, B, H, W, eps, fwd_workspace, dout,
                       dmu_sigma, grad_out, workspace, (hipStream_t)stream);
}

sv_status sv_tvae_autotune(int dtype, int factor, int B, int H, int W) {
    if (dtype != SV_F32 && dtype != SV_BF16 && dtype != SV_F16) return SV_ERR_DTYPE;
    if (factor < 1 || factor > 8) return SV_ERR_RANGE;
    if (!tv_shape_ok(factor, B, H, W)) return SV_ERR_SHAPE;
    const TvShape s = tv_shape(dtype);
    const TvLevels lv = tv_levels(factor, H, W);
    const size_t ws = sv_tvae_workspace_bytes(dtype, factor, B, H, W);
    const size_t nlow = (size_t)B * lv.h[1] * lv.w[1];
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    const size_t o_pk = take(s.bytes), o_par = take((size_t)canon_off(NCANON) * 4), o_ws = take(ws);
    const size_t o_in = take(2 * nlow), o_out = take((size_t)B * H * W * 4);
    void *mem = nullptr;
    SV_HIP(hipMalloc(&mem, off));
    char *d = (char *)mem;
    hipStream_t st = nullptr;
    // zero parameters and inputs: timing does not depend on the values
    hipLaunchKernelGGL(k_zero_bytes, dim3(4096), dim3(256), 0, st, (uint32_t *)d, off / 4);
    sv_status r = tv_pack(s, (const float *)(d + o_par), d + o_pk, st);
    const uint8_t *disp = (const uint8_t *)(d + o_in), *img = disp + nlow;
    // the configurations under test travel with each call (cur): tuning
    // changes no process-wide setting, so other threads' calls are unaffected
    int cur[T_NL], base[T_NL], best[T_NL];
    auto run = [&](int only) {
        return tv_forward(s, factor, d + o_pk, disp, img, B, H, W, nullptr, (float *)(d + o_out), nullptr,
                          d + o_ws, st, only, cur);
    };
    auto timed = [&](int only, int reps) {
        hipEvent_t a, b;
        float t = 1e30f;
        if (hipEventCreate(&a) != hipSuccess) return t;
        if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return t; }
        for (int i = 0; i < 2 && r == SV_OK; ++i) r = run(only);
        (void)hipEventRecord(a, st);
        for (int i = 0; i < reps && r == SV_OK; ++i) r = run(only);
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        (void)hipEventElapsedTime(&t, a, b);
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return t / reps;
    };
    for (int i = 0; i < T_NL; ++i) {
        const int k = kOutLevel[i];
        base[i] = tv_heuristic_cfg(i, B, lv.h[k], lv.w[k]);
        best[i] = cur[i] = base[i];
    }
    const int reps = B >= 16 ? 4 : 12;
    for (int li = 0; li < T_NL && r == SV_OK; ++li) {
        if (li == T_FE) continue;  // a direct stencil, no tile configuration
        const int dt = li == T_YP ? SV_F32 : dtype;
        const int k = kOutLevel[li];
        const long long npix = (long long)B * lv.h[k] * lv.w[k];
        float bt = 1e30f;
        best[li] = base[li];
        for (int c = 0; c < conv_num_cfgs() && r == SV_OK; ++c) {
            if (conv_resolve_cfg(dt, kLayers[li].k, kLayers[li].stride, c) != c) continue;
            // a split the launch would not take duplicates a smaller one
            const int want = c / conv_num_tiles() + 1;
            static float dummy;
            const TvAct a = tv_act(s.es, lv, B);
            if (conv_effective_split(dt, c, kLayers[li].cin, npix, s.n_pad[li], &dummy, a.part_bytes) != want) continue;
            cur[li] = c;
            const float t = timed(li, reps);
            if (t < bt) { bt = t; best[li] = c; }
        }
        cur[li] = base[li];
    }
    if (r == SV_OK) {
        // keep the tuned set only if the whole pass is faster than the defaults
        const float t0 = timed(-1, reps);
        for (int i = 0; i < T_NL; ++i) cur[i] = best[i];
        const float t1 = timed(-1, reps);
        std::lock_guard<std::mutex> g(g_tv_mu);
        if (t1 < t0) {
            std::array<int, T_NL> a;
            for (int i = 0; i < T_NL; ++i) a[i] = best[i];
            g_tv_tuned[std::make_tuple(dtype, factor, B, H, W)] = a;
        } else {
            g_tv_tuned.erase(std::make_tuple(dtype, factor, B, H, W));
        }
    }
    const hipError_t e = hipFree(mem);
    if (r == SV_OK && e != hipSuccess) r = hip_fail(e, "hipFree");
    return r;
}

sv_status sv_tvae_layer_cfgs(int dtype, int factor, int B, int H, int W, int *cfg_out) {
    if (!cfg_out) return SV_ERR_NULL;
    if (dtype != SV_F32 && dtype != SV_BF16 && dtype != SV_F16) return SV_ERR_DTYPE;
    if (factor < 1 || factor > 8) return SV_ERR_RANGE;
    if (!tv_shape_ok(factor, B, H, W)) return SV_ERR_SHAPE;
    tv_layer_cfgs(dtype, factor, B, H, W, cfg_out);
    return SV_OK;
}

}  // extern "C"
