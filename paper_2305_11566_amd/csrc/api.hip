// C ABI of libsv.so: argument validation (no HIP call before it passes) and
// dispatch to the launchers.
#include <string.h>

#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <string>

#include "net.h"
#include "prof.h"

namespace sv {

static thread_local std::string t_last_error;

sv_status hip_fail(hipError_t e, const char *where) {
    t_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return SV_ERR_HIP;
}

}  // namespace sv

using namespace sv;

extern "C" {

const char *sv_status_str(sv_status s) {
    switch (s) {
    case SV_OK: return "SV_OK";
    case SV_ERR_NULL: return "SV_ERR_NULL";
    case SV_ERR_SHAPE: return "SV_ERR_SHAPE";
    case SV_ERR_RANGE: return "SV_ERR_RANGE";
    case SV_ERR_DTYPE: return "SV_ERR_DTYPE";
    case SV_ERR_WORKSPACE: return "SV_ERR_WORKSPACE";
    case SV_ERR_UNSUPPORTED: return "SV_ERR_UNSUPPORTED";
    case SV_ERR_HIP: return "SV_ERR_HIP";
    default: return "SV_ERR_UNKNOWN";
    }
}

const char *sv_last_error(void) { return t_last_error.c_str(); }

static const int kMaxSide = 16384;

static sv_status check_window(int win_w, int win_h) {
    if (win_w < 1 || win_h < 1 || win_w % 2 == 0 || win_h % 2 == 0) return SV_ERR_RANGE;
    if (win_w > 17 || win_h > 17) return SV_ERR_RANGE;
    if (win_w * win_h - 1 > 64 || win_w * win_h - 1 < 1) return SV_ERR_RANGE;
    return SV_OK;
}

sv_status sv_census(const uint8_t *img, int B, int H, int W, int pitch, int factor, int win_w,
                    int win_h, uint8_t *low_out, uint64_t *census_out, void *stream) {
    if (!img || !census_out) return SV_ERR_NULL;
    if (B <= 0 || H <= 0 || W <= 0 || pitch < W || H > kMaxSide || W > kMaxSide) return SV_ERR_SHAPE;
    if (factor < 1 || factor > 8) return SV_ERR_RANGE;
    sv_status r = check_window(win_w, win_h);
    if (r != SV_OK) return r;
    prof_mark(PROF_CENSUS, 0, (hipStream_t)stream);
    for (int rep = prof_repeat(); rep > 0 && r == SV_OK; --rep)
        r = launch_reduce_census(img, nullptr, B, H, W, pitch, factor, win_w, win_h, low_out, nullptr,
                                 census_out, nullptr, (hipStream_t)stream);
    prof_mark(PROF_CENSUS, 1, (hipStream_t)stream);
    return r;
}

// Both views in one launch (the left view's reduced image is written when
// low_left is non-NULL).  Same contract as sv_census.
sv_status sv_census_pair(const uint8_t *left, const uint8_t *right, int B, int H, int W,
                         int pitch, int factor, int win_w, int win_h, uint8_t *low_left,
                         uint64_t *cen_left, uint64_t *cen_right, void *stream) {
    if (!left || !right || !cen_left || !cen_right) return SV_ERR_NULL;
    if (B <= 0 || H <= 0 || W <= 0 || pitch < W || H > kMaxSide || W > kMaxSide) return SV_ERR_SHAPE;
    if (factor < 1 || factor > 8) return SV_ERR_RANGE;
    sv_status r = check_window(win_w, win_h);
    if (r != SV_OK) return r;
    prof_mark(PROF_CENSUS, 0, (hipStream_t)stream);
    for (int rep = prof_repeat(); rep > 0 && r == SV_OK; --rep)
        r = launch_reduce_census(left, right, B, H, W, pitch, factor, win_w, win_h, low_left, nullptr,
                                 cen_left, cen_right, (hipStream_t)stream);
    prof_mark(PROF_CENSUS, 1, (hipStream_t)stream);
    return r;
}

}  // extern "C"

// Lanes per pixel of the cost + WTA kernel: an explicit setting
// (sv_set_cost_wta_split), else the split the autotuner measured fastest for
// this (B, h, w, D) in this process, else 4.  The result never depends on it.
static std::atomic<int> g_dsplit_override{0};
static std::mutex g_dsplit_mu;
static std::map<std::array<int, 4>, int> g_dsplit_tuned;

namespace sv {
int cost_wta_split_for(int B, int h, int w, int D) {
    const int ov = g_dsplit_override.load();
    if (ov > 0) return ov;
    std::lock_guard<std::mutex> lk(g_dsplit_mu);
    auto it = g_dsplit_tuned.find({B, h, w, D});
    return it != g_dsplit_tuned.end() ? it->second : 4;
}
void cost_wta_split_tuned(int B, int h, int w, int D, int d) {
    if (d != 1 && d != 2 && d != 4 && d != 8) return;
    std::lock_guard<std::mutex> lk(g_dsplit_mu);
    g_dsplit_tuned[{B, h, w, D}] = d;
}
int cost_wta_split_override() { return g_dsplit_override.load(); }
}  // namespace sv

extern "C" {

sv_status sv_cost_wta(const uint64_t *cen_l, const uint64_t *cen_r, int B, int h, int w, int D,
                      int nbits, uint8_t *disp_out, void *stream) {
    if (!cen_l || !cen_r || !disp_out) return SV_ERR_NULL;
    if (B <= 0 || h <= 0 || w <= 0 || h > kMaxSide || w > kMaxSide) return SV_ERR_SHAPE;
    if (D < 1 || D > 256 || nbits < 1 || nbits > 64) return SV_ERR_RANGE;
    prof_mark(PROF_COST_WTA, 0, (hipStream_t)stream);
    const int dsplit = cost_wta_split_for(B, h, w, D);
    sv_status r = SV_OK;
    for (int rep = prof_repeat(); rep > 0 && r == SV_OK; --rep)
        r = launch_cost_wta(cen_l, cen_r, B, h, w, D, nbits, disp_out, dsplit, (hipStream_t)stream);
    prof_mark(PROF_COST_WTA, 1, (hipStream_t)stream);
    return r;
}

size_t sv_sgm_workspace_bytes(int B, int h, int w, int D) {
    if (B <= 0 || h <= 0 || w <= 0 || D <= 0) return 0;
    return sgm_volume_bytes(B, h, w, D);
}

sv_status sv_sgm(const uint64_t *cen_l, const uint64_t *cen_r, int B, int h, int w, int D, int nbits,
                 int P1, int P2, uint8_t *disp_out, void *workspace, size_t ws_bytes, void *stream) {
    if (!cen_l || !cen_r || !disp_out || !workspace) return SV_ERR_NULL;
    if (B <= 0 || h <= 0 || w <= 0 || h > kMaxSide || w > kMaxSide) return SV_ERR_SHAPE;
    if (D < 1 || D > 256 || nbits < 1 || nbits > 64) return SV_ERR_RANGE;
    if (P1 < 0 || P2 < P1 || nbits + 1 + P2 > 255) return SV_ERR_RANGE;
    if (ws_bytes < sv_sgm_workspace_bytes(B, h, w, D)) return SV_ERR_WORKSPACE;
    return launch_sgm(cen_l, cen_r, B, h, w, D, nbits, P1, P2, (uint8_t *)workspace, disp_out,
                      (hipStream_t)stream);
}

static sv_status check_zncc(const uint8_t *ll, const uint8_t *lr, const void *out, int B, int h,
                            int w, int D, int win_w, int win_h) {
    if (!ll || !lr || !out) return SV_ERR_NULL;
    if (B <= 0 || h <= 0 || w <= 0 || h > kMaxSide || w > kMaxSide) return SV_ERR_SHAPE;
    if (D < 1 || D > 256) return SV_ERR_RANGE;
    if (win_w < 1 || win_h < 1 || win_w % 2 == 0 || win_h % 2 == 0 || win_w > 17 || win_h > 17)
        return SV_ERR_RANGE;
    return SV_OK;
}

sv_status sv_zncc_sgm(const uint8_t *low_l, const uint8_t *low_r, int B, int h, int w, int D,
                      int win_w, int win_h, int P1, int P2, uint8_t *disp_out, void *workspace,
                      size_t ws_bytes, void *stream) {
    sv_status r = check_zncc(low_l, low_r, disp_out, B, h, w, D, win_w, win_h);
    if (r != SV_OK) return r;
    if (!workspace) return SV_ERR_NULL;
    if (P1 < 0 || P2 < P1 || 64 + P2 > 255) return SV_ERR_RANGE;
    if (ws_bytes < sv_sgm_workspace_bytes(B, h, w, D)) return SV_ERR_WORKSPACE;
    return launch_zncc_sgm(low_l, low_r, B, h, w, D, win_w, win_h, P1, P2, (uint8_t *)workspace,
                           disp_out, (hipStream_t)stream);
}

sv_status sv_zncc_cost(const uint8_t *low_l, const uint8_t *low_r, int B, int h, int w, int D,
                       int win_w, int win_h, uint8_t *cost_out, void *stream) {
    sv_status r = check_zncc(low_l, low_r, cost_out, B, h, w, D, win_w, win_h);
    if (r != SV_OK) return r;
    return launch_zncc_cost(low_l, low_r, B, h, w, D, D, win_w, win_h, cost_out, (hipStream_t)stream);
}

size_t sv_smp_workspace_bytes(int B, int h, int w) {
    if (B <= 0 || h <= 0 || w <= 0) return 0;
    return (size_t)B * h * w;
}

sv_status sv_smp_median(const uint8_t *disp_in, int B, int h, int w, int D, uint8_t *disp_out,
                        void *workspace, size_t ws_bytes, void *stream) {
    if (!disp_in || !disp_out || !workspace) return SV_ERR_NULL;
    if (B <= 0 || h <= 0 || w <= 0 || h > kMaxSide || w > 16384) return SV_ERR_SHAPE;
    if (D < 1 || D > 256) return SV_ERR_RANGE;
    if (ws_bytes < sv_smp_workspace_bytes(B, h, w)) return SV_ERR_WORKSPACE;
    return launch_smp_median(disp_in, B, h, w, D, (uint8_t *)workspace, disp_out,
                             (hipStream_t)stream);
}

// Lanes per pixel of the cost + WTA kernel (1, 2, 4 or 8; 0 restores the
// per-shape choice); for tuning and tests.
sv_status sv_set_cost_wta_split(int dsplit) {
    if (dsplit != 0 && dsplit != 1 && dsplit != 2 && dsplit != 4 && dsplit != 8) return SV_ERR_RANGE;
    g_dsplit_override.store(dsplit);
    return SV_OK;
}

int64_t sv_vae_param_count(const sv_vae_desc *desc) {
    NetShape ns;
    sv_status r = net_shape(desc, ns);
    return r == SV_OK ? ns.nparams : (int64_t)r;
}

size_t sv_vae_packed_bytes(const sv_vae_desc *desc) {
    NetShape ns;
    return net_shape(desc, ns) == SV_OK ? ns.packed_bytes : 0;
}

sv_status sv_vae_pack_weights(const sv_vae_desc *desc, const float *params, void *packed_out,
                              void *stream) {
    NetShape ns;
    sv_status r = net_shape(desc, ns);
    if (r != SV_OK) return r;
    if (!params || !packed_out) return SV_ERR_NULL;
    if ((uintptr_t)packed_out % 256) return SV_ERR_RANGE;
    return net_pack(ns, params, packed_out, (hipStream_t)stream);
}

static bool shape_ok(int B, int H, int W) {
    return B > 0 && H > 0 && W > 0 && H <= kMaxSide && W <= kMaxSide && (int64_t)B * H * W < (1ll << 31);
}

size_t sv_vae_workspace_bytes(const sv_vae_desc *desc, int B, int H, int W) {
    NetShape ns;
    if (net_shape(desc, ns) != SV_OK || !shape_ok(B, H, W)) return 0;
    const Levels lv = net_levels(ns, H, W);
    const ActLayout a = net_act_layout(ns, lv, B);
    const size_t fwd = a.ws_fwd + a.saved;
    const size_t bwd = a.ws_fwd + net_bwd_workspace(ns, lv, B);
    return fwd > bwd ? fwd : bwd;
}

size_t sv_vae_saved_bytes(const sv_vae_desc *desc, int B, int H, int W) {
    NetShape ns;
    if (net_shape(desc, ns) != SV_OK || !shape_ok(B, H, W)) return 0;
    return net_act_layout(ns, net_levels(ns, H, W), B).saved;
}

sv_status sv_vae_forward(const sv_vae_desc *desc, const void *packed_w, const uint8_t *disp_low,
                         const uint8_t *img_low, int B, int H, int W, const float *eps, float *out,
                         float *mu_logvar, void *saved, void *workspace, size_t ws_bytes,
                         void *stream) {
    NetShape ns;
    sv_status r = net_shape(desc, ns);
    if (r != SV_OK) return r;
    if (!packed_w || !disp_low || !img_low || !out || !workspace) return SV_ERR_NULL;
    if (eps && !saved) return SV_ERR_NULL;   // sampling z is only for training
    if (ns.dtype == SV_I8 && (eps || saved)) return SV_ERR_UNSUPPORTED;  // INT8: inference only
    if (!shape_ok(B, H, W)) return SV_ERR_SHAPE;
    if (ws_bytes < sv_vae_workspace_bytes(desc, B, H, W)) return SV_ERR_WORKSPACE;
    if ((uintptr_t)workspace % 256 || (saved && (uintptr_t)saved % 256) || (uintptr_t)packed_w % 256)
        return SV_ERR_RANGE;
    if (mu_logvar && (uintptr_t)mu_logvar % 16) return SV_ERR_RANGE;
    return net_forward(ns, packed_w, disp_low, img_low, B, H, W, eps, out, mu_logvar, saved,
                       workspace, (hipStream_t)stream);
}

sv_status sv_vae_backward(const sv_vae_desc *desc, const void *packed_w, const void *saved,
                          int B, int H, int W, const float *eps, const float *dout,
                          const float *dmu_logvar, float kl_weight, float *grad_out,
                          void *workspace, size_t ws_bytes, void *stream) {
    NetShape ns;
    sv_status r = net_shape(desc, ns);
    if (r != SV_OK) return r;
    if (ns.dtype == SV_I8) return SV_ERR_UNSUPPORTED;
    if (!packed_w || !saved || !dout || !grad_out || !workspace) return SV_ERR_NULL;
    if (!shape_ok(B, H, W)) return SV_ERR_SHAPE;
    if (ws_bytes < sv_vae_workspace_bytes(desc, B, H, W)) return SV_ERR_WORKSPACE;
    if ((uintptr_t)workspace % 256 || (uintptr_t)saved % 256 || (uintptr_t)packed_w % 256)
        return SV_ERR_RANGE;
    return net_backward(ns, packed_w, saved, B, H, W, eps, dout, dmu_logvar, kl_weight, grad_out,
                        workspace, (hipStream_t)stream);
}

// Selects the tile configuration of one network layer (0..8; -1 = default)
// for every compute dtype.
sv_status sv_set_layer_cfg(int layer, int cfg) {
    if (layer < 0 || layer >= NLAYERS) return SV_ERR_RANGE;
    if (cfg < -1 || cfg >= conv_num_cfgs()) return SV_ERR_RANGE;
    for (int dt = 0; dt < 4; ++dt) net_set_cfg_override(dt, layer, cfg);
    return SV_OK;
}

int sv_num_layer_cfgs(void) { return conv_num_cfgs(); }

sv_status sv_set_latent_fusion(int on) {
    if (on != 0 && on != 1) return SV_ERR_RANGE;
    net_set_latent_fusion(on);
    return SV_OK;
}

}  // extern "C"
