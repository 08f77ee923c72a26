// Host-side runner of the refinement network's forward pass (Table I in the
// shape described in sv.h): one implicit-GEMM launch per layer, then the
// final gather kernel.  No host synchronisation, no allocation.
#include <algorithm>
#include <atomic>

#include "net.h"
#include "prof.h"

namespace sv {

static inline int rup(int v, int m) { return (v + m - 1) / m * m; }

sv_status net_shape(const sv_vae_desc *d, NetShape &ns) {
    if (!d) return SV_ERR_NULL;
    const int cs[4] = {d->c1, d->c2, d->c3, d->latent};
    for (int c : cs)
        if (c < 8 || c > 256 || c % 8) return SV_ERR_RANGE;
    if (d->factor < 1 || d->factor > 8) return SV_ERR_RANGE;
    if (d->dtype != SV_F32 && d->dtype != SV_BF16 && d->dtype != SV_F16 && d->dtype != SV_I8)
        return SV_ERR_DTYPE;
    ns.c1 = d->c1; ns.c2 = d->c2; ns.c3 = d->c3; ns.L = d->latent; ns.f = d->factor;
    ns.dtype = d->dtype;
    ns.es = dtype_bytes(d->dtype);
    const int c1 = ns.c1, c2 = ns.c2, c3 = ns.c3, L = ns.L;
    const LayerSpec t[NLAYERS] = {
        {c1, 2, 3, 2},      {c2, c1, 3, 2},      {c3, c2, 3, 2},
        {2 * L, c3, 1, 1},  {c3, L, 1, 1},       {c2, c3 + c2, 3, 1},
        {c1, c2 + c1, 3, 1}, {c1, c1 + 2, 3, 1}, {1, c1 + 2, 3, 1},
    };
    size_t off = 0;
    int64_t poff = 0;
    for (int i = 0; i < NLAYERS; ++i) {
        ns.ly[i] = t[i];
        ns.p_off[i] = poff;
        poff += (int64_t)t[i].cout * t[i].cin * t[i].k * t[i].k + t[i].cout;
        ns.cin_pad[i] = rup(t[i].cin, 8);
        // the final layer is packed as a 1x1 layer with one output row per tap
        ns.n_pad[i] = (i == L_F) ? 16 : rup(t[i].cout, 16);
        const int taps = (i == L_F) ? 1 : t[i].k * t[i].k;
        // the final projection stays FP32 in every mode: rounding its few weights
        // dominates the reduced-precision error of the refined map
        const bool i8 = ns.dtype == SV_I8 && i != L_F;
        const int les = (i == L_F) ? 4 : (i8 ? 1 : ns.es);
        ns.w_off[i] = off;
        off = align256(off + (size_t)taps * ns.n_pad[i] * ns.cin_pad[i] * les);
        ns.b_off[i] = off;
        off = align256(off + (size_t)t[i].cout * sizeof(float));
        ns.s_off[i] = 0;
        if (i8) {
            ns.s_off[i] = off;
            off = align256(off + (size_t)ns.n_pad[i] * sizeof(float));
        }
    }
    for (int i = 0; i < NLAYERS; ++i) {
        ns.bw_off[i] = 0;
        ns.bn_pad[i] = ns.bcin_pad[i] = 0;
        if (i == L_E1 || i == L_F || ns.dtype == SV_I8) continue;  // INT8: inference only
        ns.bn_pad[i] = rup(t[i].cin, 16);
        ns.bcin_pad[i] = rup(t[i].cout, 8);
        ns.bw_off[i] = off;
        off = align256(off + (size_t)t[i].k * t[i].k * ns.bn_pad[i] * ns.bcin_pad[i] * ns.es);
    }
    ns.packed_bytes = off;
    ns.nparams = poff;
    return SV_OK;
}

Levels net_levels(const NetShape &ns, int H, int W) {
    Levels lv;
    lv.H = H; lv.W = W;
    lv.h[0] = cdiv(H, ns.f); lv.w[0] = cdiv(W, ns.f);
    for (int k = 1; k < 4; ++k) { lv.h[k] = cdiv(lv.h[k - 1], 2); lv.w[k] = cdiv(lv.w[k - 1], 2); }
    return lv;
}

ActLayout net_act_layout(const NetShape &ns, const Levels &lv, int B) {
    ActLayout a;
    auto px = [&](int k) { return (size_t)B * lv.h[k] * lv.w[k]; };
    size_t o = 0;
    a.E1 = o; o = align256(o + px(1) * ns.c1 * ns.es);
    a.E2 = o; o = align256(o + px(2) * ns.c2 * ns.es);
    a.E3 = o; o = align256(o + px(3) * ns.c3 * ns.es);
    // partial sums of split-reduction launches: room for the largest layer
    // output at the maximum split, capped
    static const int out_level[NLAYERS] = {1, 2, 3, 3, 3, 2, 1, 0, 0};
    size_t part = 0;
    for (int i = 0; i < L_F; ++i)
        part = std::max(part, (size_t)CONV_MAX_SPLIT * px(out_level[i]) * ns.n_pad[i] * sizeof(float));
    a.part_bytes = std::min(part, CONV_PART_CAP);
    a.part = o; o = align256(o + a.part_bytes);
    a.amax = o; o = align256(o + (size_t)AM_NSLOTS * AMAX_SUB * sizeof(uint32_t));
    a.ws_fwd = o;
    o = 0;
    a.disp = o; o = align256(o + px(0));
    a.img = o;  o = align256(o + px(0));
    a.ML = o;   o = align256(o + px(3) * 2 * ns.L * sizeof(float));
    a.Z = o;    o = align256(o + px(3) * ns.L * ns.es);
    a.G3 = o;   o = align256(o + px(3) * ns.c3 * ns.es);
    a.G2 = o;   o = align256(o + px(2) * ns.c2 * ns.es);
    a.G1 = o;   o = align256(o + px(1) * ns.c1 * ns.es);
    // G0's slot: the map itself (training), or at inference the nine FP32
    // tap projections of the final layer that G0's epilogue writes instead
    a.G0 = o;   o = align256(o + px(0) * std::max<size_t>((size_t)ns.c1 * ns.es, 9 * sizeof(float)));
    a.saved = o;
    return a;
}

size_t net_infer_bytes(const NetShape &ns, const Levels &lv, int B) {
    const ActLayout a = net_act_layout(ns, lv, B);
    return a.ws_fwd + a.saved;
}

// ---- tile configuration per layer ----------------------------------------------
// per compute dtype and layer; -1 = default
static std::atomic<int> g_cfg_override[4][NLAYERS];
static struct CfgInit {
    CfgInit() {
        for (auto &d : g_cfg_override)
            for (auto &v : d) v.store(-1);
    }
} g_cfg_init;

void net_set_cfg_override(int dtype, int layer, int cfg) {
    if (dtype >= 0 && dtype < 4 && layer >= 0 && layer < NLAYERS) g_cfg_override[dtype][layer].store(cfg);
}
int net_get_cfg_override(int dtype, int layer) {
    return (dtype >= 0 && dtype < 4 && layer >= 0 && layer < NLAYERS) ? g_cfg_override[dtype][layer].load()
                                                                       : -1;
}

int net_heuristic_cfg(const NetShape &ns, int layer) {
    const int cout = layer == L_F ? 16 : ns.ly[layer].cout;
    if (cout <= 16) return 5;   // th4_tn16
    if (cout <= 32) return 2;   // th4_tn32
    return 0;                   // th4_tn64
}

bool net_projects(const NetShape &ns, bool train) {
    return !train && ns.c1 <= 64;
}

int net_g0_proj_cfg(const NetShape &ns, int cfg) {
    int c = conv_resolve_cfg(ns.dtype, 3, 1, cfg % conv_num_tiles());  // no split
    if (!conv_cfg_projects(c, ns.c1)) c = ns.c1 <= 32 ? 2 /* th4_tn32 */ : 0 /* th4_tn64 */;
    return c;
}

int net_default_cfg(const NetShape &ns, int layer, int M) {
    const int ov = net_get_cfg_override(ns.dtype, layer);
    if (ov >= 0 && ov < conv_num_cfgs()) return ov;
    (void)M;
    return net_heuristic_cfg(ns, layer);
}

void net_layer_cfgs(const NetShape &ns, int B, int H, int W, int *cfg) {
    int tuned[NLAYERS];
    const bool have = tuned_lookup(ns, B, H, W, tuned, nullptr);
    for (int i = 0; i < NLAYERS; ++i) {
        const int ov = net_get_cfg_override(ns.dtype, i);
        cfg[i] = ov >= 0 ? ov : (have ? tuned[i] : net_default_cfg(ns, i, 0));
        if (i < L_F) cfg[i] = conv_resolve_cfg(ns.dtype, ns.ly[i].k, ns.ly[i].stride, cfg[i]);
    }
}

// The reduction split layer `layer` gets from configuration cfg in a forward
// pass of batch B at H x W (1: no split).
int net_layer_split(const NetShape &ns, int layer, int cfg, int B, int H, int W) {
    if (layer < 0 || layer >= L_F) return 1;
    static const int out_level[NLAYERS] = {1, 2, 3, 3, 3, 2, 1, 0, 0};
    const Levels lv = net_levels(ns, H, W);
    const ActLayout a = net_act_layout(ns, lv, B);
    const int k = out_level[layer];
    const long long npix = (long long)B * lv.h[k] * lv.w[k];
    const int dt = ns.dtype;
    static float dummy;
    return conv_effective_split(dt, cfg, ns.ly[layer].cin, npix, ns.n_pad[layer], &dummy, a.part_bytes);
}

// ---- forward ------------------------------------------------------------------------
static ConvSrc src_tensor(const void *p, int C, int pitch, int coff, int hs, int ws, int sdt) {
    ConvSrc s{};
    s.ptr = p; s.kind = SRC_TENSOR; s.C = C; s.pitch = pitch; s.coff = coff; s.hs = hs; s.ws = ws;
    s.sdt = sdt;
    return s;
}
static ConvSrc src_resize(const void *p, int C, int hs, int ws) {
    ConvSrc s = src_tensor(p, C, C, 0, hs, ws, 0);
    s.kind = SRC_RESIZE;
    return s;
}
static ConvSrc src_x0(const uint8_t *disp, const uint8_t *img, int hs, int ws, int f) {
    ConvSrc s{};
    s.ptr = disp; s.img = img; s.kind = SRC_X0; s.C = 2; s.hs = hs; s.ws = ws;
    s.scale0 = (float)f / 256.0f;
    return s;
}

// INT8 passes: the amax slots of the layer's sources and output
struct LayerAmax { const uint32_t *in0, *in1; uint32_t *out; };

static ConvParams layer_params(const NetShape &ns, const void *packed, int li, ConvSrc s0, ConvSrc s1,
                               int B, int Hi, int Wi, int Ho, int Wo, void *out, int out_pitch,
                               int out_f32, int act, float *part, size_t part_bytes, LayerAmax am) {
    ConvParams p{};
    if (ns.dtype == SV_I8 && li != L_F) {
        p.wscale = (const float *)((const char *)packed + ns.s_off[li]);
        p.amax_in[0] = am.in0;
        p.amax_in[1] = am.in1;
    }
    p.amax_out = am.out;
    p.part = part;
    p.part_bytes = part_bytes;
    p.src[0] = s0; p.src[1] = s1;
    p.B = B; p.Hi = Hi; p.Wi = Wi; p.Ho = Ho; p.Wo = Wo;
    p.Cin = s0.C + (s1.kind ? s1.C : 0);
    const bool tsplit = li == L_F;
    p.Cout = tsplit ? 9 : ns.ly[li].cout;
    p.cin_pad = ns.cin_pad[li];
    p.n_pad = ns.n_pad[li];
    p.wpk = (const char *)packed + ns.w_off[li];
    p.bias = tsplit ? nullptr : (const float *)((const char *)packed + ns.b_off[li]);
    p.out = out; p.out_pitch = out_pitch; p.out_coff = 0;
    p.act = act; p.out_f32 = out_f32;
    return p;
}

// A layer's launch; a split reduction leaves its partial sums for the
// second pass, which the caller runs after the layer's profiling stage
// (recorded as a stage of its own, see SplitSum).
struct SplitSum {
    ConvParams p;
    int dtype = 0, ksplit = 1;
};

static sv_status run_layer(const NetShape &ns, const void *packed, int li, ConvSrc s0, ConvSrc s1,
                           int B, int Hi, int Wi, int Ho, int Wo, void *out, int out_pitch,
                           int out_f32, int act, int cfg, float *part, size_t part_bytes,
                           LayerAmax am, hipStream_t st, SplitSum *ss) {
    ConvParams p = layer_params(ns, packed, li, s0, s1, B, Hi, Wi, Ho, Wo, out, out_pitch,
                                out_f32, act, part, part_bytes, am);
    p.defer_sum = 1;
    const bool tsplit = li == L_F;
    const int ks = tsplit ? 1 : ns.ly[li].k;
    const int stride = tsplit ? 1 : ns.ly[li].stride;
    ss->p = p;
    ss->dtype = tsplit ? SV_F32 : ns.dtype;
    return launch_conv_split(ss->dtype, ks, stride, cfg, p, st, &ss->ksplit);
}

// The second pass of a split layer, as profiling stage PROF_SPLIT.
static sv_status run_split_sum(const SplitSum &ss, hipStream_t st) {
    if (ss.ksplit <= 1) return SV_OK;
    prof_mark(PROF_SPLIT, 0, st);
    sv_status r = SV_OK;
    for (int rep = prof_repeat(); rep > 0 && r == SV_OK; --rep) r = launch_split_sum(ss.dtype, ss.p, ss.ksplit, st);
    prof_mark(PROF_SPLIT, 1, st);
    return r;
}

// 1: an inference pass runs the head and G3 as one kernel where the shapes allow
static std::atomic<int> g_latent_fusion{1};
void net_set_latent_fusion(int on) { g_latent_fusion.store(on ? 1 : 0); }

// with only >= 0, a forward pass launches that layer alone (the autotuner
// times one layer at a time on buffers a full pass has filled)
template <typename... A>
static sv_status run_layer_if(int only, const NetShape &ns, const void *packed, int li, A... args) {
    if (only >= 0 && only != li) return SV_OK;
    return run_layer(ns, packed, li, args...);
}
// a layer (profiling stage ev) and then its split sum (stage PROF_SPLIT)
#define SV_LAYER(ev, li, ...)                                                     \
    do {                                                                          \
        SplitSum ss_;                                                             \
        ev_rec(ev, 0, st);                                                        \
        SV_STAGE(run_layer_if(only, ns, packed, li, __VA_ARGS__, st, &ss_));      \
        ev_rec(ev, 1, st);                                                        \
        if (only < 0 || only == li) SV_TRY(run_split_sum(ss_, st));               \
    } while (0)

// launch i of the forward pass is profiling stage PROF_E1 + i
static inline void ev_rec(int i, int which, hipStream_t st) { prof_mark(PROF_E1 + i, which, st); }

#define SV_TRY(x)                       \
    do {                                \
        sv_status r_ = (x);             \
        if (r_ != SV_OK) return r_;     \
    } while (0)

// a profiled stage: launched prof_repeat() times back to back (once unless
// profiling asks for repeats)
#define SV_STAGE(x) \
    for (int rep_ = prof_repeat(); rep_ > 0; --rep_) SV_TRY(x)

sv_status net_forward(const NetShape &ns, const void *packed, const uint8_t *disp,
                      const uint8_t *img, int B, int H, int W, const float *eps, float *out,
                      float *ml_user, void *saved, void *ws, hipStream_t st, int only,
                      const int *cfg_in) {
    const Levels lv = net_levels(ns, H, W);
    const ActLayout a = net_act_layout(ns, lv, B);
    int cfg[NLAYERS];
    if (cfg_in) {
        for (int i = 0; i < NLAYERS; ++i)
            cfg[i] = i < L_F ? conv_resolve_cfg(ns.dtype, ns.ly[i].k, ns.ly[i].stride, cfg_in[i]) : cfg_in[i];
    } else {
        net_layer_cfgs(ns, B, H, W, cfg);
    }
    char *w = (char *)ws;
    const bool train = saved != nullptr;                   // keep what the backward needs
    char *sv_ = train ? (char *)saved : w + a.ws_fwd;      // else it lives in the workspace
    void *E1 = w + a.E1, *E2 = w + a.E2, *E3 = w + a.E3;
    float *part = (float *)(w + a.part);
    float *ML = (!train && ml_user) ? ml_user : (float *)(sv_ + a.ML);
    void *Z = sv_ + a.Z, *G3 = sv_ + a.G3, *G2 = sv_ + a.G2, *G1 = sv_ + a.G1, *G0 = sv_ + a.G0;
    const int c1 = ns.c1, c2 = ns.c2, c3 = ns.c3, L = ns.L;
    const ConvSrc none{};

    if (train) {  // keep the coarse inputs for the backward pass
        const size_t n0 = (size_t)B * lv.h[0] * lv.w[0];
        SV_HIP(hipMemcpyAsync(sv_ + a.disp, disp, n0, hipMemcpyDeviceToDevice, st));
        SV_HIP(hipMemcpyAsync(sv_ + a.img, img, n0, hipMemcpyDeviceToDevice, st));
    }
    const ConvSrc x0 = src_x0(disp, img, lv.h[0], lv.w[0], ns.f);
    // INT8: per-tensor amax slots, cleared, and x0's recorded, before the layers
    const bool q8 = ns.dtype == SV_I8;
    uint32_t *AM = q8 ? (uint32_t *)(w + a.amax) : nullptr;
    auto am = [&](int i0, int i1, int o) {
        auto slot = [&](int k) -> uint32_t * { return (AM && k >= 0) ? AM + (size_t)k * AMAX_SUB : nullptr; };
        return LayerAmax{slot(i0), slot(i1), slot(o)};
    };
    if (q8)
        SV_TRY(launch_amax_prologue(AM, AM_NSLOTS, AM_X0, disp, img, (long long)B * lv.h[0] * lv.w[0],
                                    (float)ns.f / 256.0f, st));
    // encoder; E1 reads the two x0 channels only: a direct stencil (INT8: on
    // the quantised layer's codes, with exact integer sums)
    ev_rec(0, 0, st);
    if (only < 0 || only == L_E1) {
        const LayerAmax a1 = am(AM_X0, -1, AM_E1);
        SV_STAGE(launch_enc1(ns.dtype, disp, img, (float)ns.f / 256.0f, B, lv.h[0], lv.w[0], lv.h[1], lv.w[1], c1,
                             (const char *)packed + ns.w_off[L_E1], ns.n_pad[L_E1], ns.cin_pad[L_E1],
                             (const float *)((const char *)packed + ns.b_off[L_E1]), E1, st,
                             q8 ? (const float *)((const char *)packed + ns.s_off[L_E1]) : nullptr, a1.in0,
                             a1.out));
    }
    ev_rec(0, 1, st);
    SV_LAYER(1, L_E2, src_tensor(E1, c1, c1, 0, lv.h[1], lv.w[1], 0), none, B, lv.h[1], lv.w[1], lv.h[2], lv.w[2],
             E2, c2, 0, 1, cfg[L_E2], part, a.part_bytes, am(AM_E1, -1, AM_E2));
    // inference: the head and G3 run as one kernel, which also finishes E3's
    // split sum when E3 runs split (E3 is then never stored)
    const bool fuse_latent = only < 0 && !eps && !train && g_latent_fusion.load() && latent_fusable(ns.dtype, c3, L);
    int e3split = 1;
    if (fuse_latent) {
        ConvParams p3 = layer_params(ns, packed, L_E3, src_tensor(E2, c2, c2, 0, lv.h[2], lv.w[2], 0), none, B,
                                     lv.h[2], lv.w[2], lv.h[3], lv.w[3], E3, c3, 0, 1, part, a.part_bytes,
                                     LayerAmax{});
        p3.defer_sum = 1;
        ev_rec(2, 0, st);
        SV_STAGE(launch_conv_split(ns.dtype, ns.ly[L_E3].k, ns.ly[L_E3].stride, cfg[L_E3], p3, st, &e3split));
        ev_rec(2, 1, st);
    } else {
        SV_LAYER(2, L_E3, src_tensor(E2, c2, c2, 0, lv.h[2], lv.w[2], 0), none, B, lv.h[2], lv.w[2], lv.h[3],
                 lv.w[3], E3, c3, 0, 1, cfg[L_E3], part, a.part_bytes, am(AM_E2, -1, AM_E3));
    }
    // latent head -> [mu | logvar] in FP32
    const ConvSrc e3src = src_tensor(E3, c3, c3, 0, lv.h[3], lv.w[3], 0);
    const ConvSrc musrc = src_tensor(ML, L, 2 * L, 0, lv.h[3], lv.w[3], SDT_F32);  // z = mu
    if (fuse_latent) {
        // inference: head and G3 in one launch (profiled as the head's stage)
        const int h3 = lv.h[3], w3 = lv.w[3];
        const ConvParams ph = layer_params(ns, packed, L_HEAD, e3src, none, B, h3, w3, h3, w3, ML, 2 * L,
                                           1, 0, nullptr, 0, LayerAmax{});
        const ConvParams pg = layer_params(ns, packed, L_G3, musrc, none, B, h3, w3, h3, w3, G3, c3, 0,
                                           1, nullptr, 0, LayerAmax{});
        ev_rec(3, 0, st);
        const float *e3bias = (const float *)((const char *)packed + ns.b_off[L_E3]);
        SV_STAGE(launch_latent(ns.dtype, ph, pg, B * h3 * w3, part, e3split, e3bias, st));
        ev_rec(3, 1, st);
    } else {
        SV_LAYER(3, L_HEAD, e3src, none, B, lv.h[3], lv.w[3], lv.h[3], lv.w[3], ML, 2 * L, 1, 0, cfg[L_HEAD],
                 part, a.part_bytes, am(AM_E3, -1, AM_ML));
        ConvSrc zsrc = musrc;
        if (eps) {
            ev_rec(4, 0, st);
            if (only < 0) SV_STAGE(launch_reparam(ML, eps, B * lv.h[3] * lv.w[3], L, Z, ns.dtype, st));
            ev_rec(4, 1, st);
            zsrc = src_tensor(Z, L, L, 0, lv.h[3], lv.w[3], 0);
        }
        // decoder
        SV_LAYER(5, L_G3, zsrc, none, B, lv.h[3], lv.w[3], lv.h[3], lv.w[3], G3, c3, 0, 1, cfg[L_G3], part,
                 a.part_bytes, am(AM_ML, -1, AM_G3));
    }
    SV_LAYER(6, L_G2, src_resize(G3, c3, lv.h[3], lv.w[3]), src_tensor(E2, c2, c2, 0, lv.h[2], lv.w[2], 0), B,
             lv.h[2], lv.w[2], lv.h[2], lv.w[2], G2, c2, 0, 1, cfg[L_G2], part, a.part_bytes,
             am(AM_G3, AM_E2, AM_G2));
    SV_LAYER(7, L_G1, src_resize(G2, c2, lv.h[2], lv.w[2]), src_tensor(E1, c1, c1, 0, lv.h[1], lv.w[1], 0), B,
             lv.h[1], lv.w[1], lv.h[1], lv.w[1], G1, c1, 0, 1, cfg[L_G1], part, a.part_bytes,
             am(AM_G2, AM_E1, AM_G1));
    // G0; at inference its epilogue writes the final layer's nine per-tap
    // projections of [G0, x0] (FP32) in place of the map, and the final layer
    // is the gather alone
    const bool proj = net_projects(ns, train);
    const float *wF = (const float *)((const char *)packed + ns.w_off[L_F]);
    const long long plane0 = (long long)B * lv.h[0] * lv.w[0];
    if (proj) {
        ev_rec(8, 0, st);
        if (only < 0 || only == L_G0) {
            ConvParams p = layer_params(ns, packed, L_G0, src_resize(G1, c1, lv.h[1], lv.w[1]), x0, B, lv.h[0],
                                        lv.w[0], lv.h[0], lv.w[0], G0, c1, 0, 1, part, a.part_bytes,
                                        am(AM_G1, AM_X0, -1));
            p.proj_w = wF;
            p.proj_pitch = ns.cin_pad[L_F];
            p.proj_out = (float *)G0;
            p.proj_plane = plane0;
            p.proj_disp = disp;
            p.proj_img = img;
            p.proj_scale0 = (float)ns.f / 256.0f;
            SV_STAGE(launch_conv(ns.dtype, 3, 1, net_g0_proj_cfg(ns, cfg[L_G0]), p, st));
        }
        ev_rec(8, 1, st);
    } else {
        SV_LAYER(8, L_G0, src_resize(G1, c1, lv.h[1], lv.w[1]), x0, B, lv.h[0], lv.w[0], lv.h[0], lv.w[0], G0, c1,
                 0, 1, cfg[L_G0], part, a.part_bytes, am(AM_G1, AM_X0, -1));
    }
    // final layer: the gather of the projections (inference), or projections
    // of the stored [G0, x0] and the gather in one kernel
    const float *biasF = (const float *)((const char *)packed + ns.b_off[L_F]);
    ev_rec(10, 0, st);
    if (only < 0) {
        if (proj)
            SV_STAGE(launch_final_gather((const float *)G0, plane0, disp, ns.f, biasF, B, lv.h[0], lv.w[0], H, W,
                                       out, st));
        else
            SV_STAGE(launch_final(q8 ? SV_BF16 : ns.dtype, G0, c1, disp, img, wF, ns.cin_pad[L_F], ns.f, biasF, B,
                                lv.h[0], lv.w[0], H, W, out, st));
    }
    ev_rec(10, 1, st);
    if (train && ml_user)
        SV_HIP(hipMemcpyAsync(ml_user, ML, (size_t)B * lv.h[3] * lv.w[3] * 2 * L * sizeof(float),
                              hipMemcpyDeviceToDevice, st));
    return SV_OK;
}

sv_status net_pack(const NetShape &ns, const float *params, void *packed, hipStream_t st) {
    for (int i = 0; i < NLAYERS; ++i) {
        const LayerSpec &l = ns.ly[i];
        const float *w = params + ns.p_off[i];
        if (ns.dtype == SV_I8 && i != L_F)
            SV_TRY(launch_pack_i8(w, l.cout, l.cin, l.k, ns.n_pad[i], ns.cin_pad[i],
                                  (int8_t *)((char *)packed + ns.w_off[i]),
                                  (float *)((char *)packed + ns.s_off[i]), st));
        else
            SV_TRY(launch_pack(i == L_F ? SV_F32 : ns.dtype, w, l.cout, l.cin, l.k, ns.n_pad[i],
                               ns.cin_pad[i], i == L_F ? 1 : 0, (char *)packed + ns.w_off[i], st));
        if (ns.bw_off[i])
            SV_TRY(launch_pack(ns.dtype, w, l.cout, l.cin, l.k, ns.bn_pad[i], ns.bcin_pad[i], 2,
                               (char *)packed + ns.bw_off[i], st));
        const float *b = w + (size_t)l.cout * l.cin * l.k * l.k;
        SV_HIP(hipMemcpyAsync((char *)packed + ns.b_off[i], b, sizeof(float) * l.cout,
                              hipMemcpyDeviceToDevice, st));
    }
    return SV_OK;
}

}  // namespace sv
