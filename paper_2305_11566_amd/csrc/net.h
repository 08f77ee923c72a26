// Shape bookkeeping of the refinement network: layer table, level sizes,
// packed-weight layout and activation layout (host side).
#pragma once

#include "kernels.h"

namespace sv {

enum Layer { L_E1 = 0, L_E2, L_E3, L_HEAD, L_G3, L_G2, L_G1, L_G0, L_F, NLAYERS };

struct LayerSpec { int cout, cin, k, stride; };

struct NetShape {
    int c1, c2, c3, L, f, dtype, es;  // es: bytes per stored element of the compute dtype
    LayerSpec ly[NLAYERS];
    int n_pad[NLAYERS], cin_pad[NLAYERS];
    size_t w_off[NLAYERS], b_off[NLAYERS], packed_bytes;
    size_t s_off[NLAYERS];  // INT8: per-row weight scales (FP32 [n_pad]); 0 otherwise
    // adjoint weights (rows = the layer's inputs, columns = its outputs, kernel
    // flipped) for the layers whose input gradient is needed
    int bn_pad[NLAYERS], bcin_pad[NLAYERS];
    size_t bw_off[NLAYERS];  // 0 when absent (E1, F)
    int64_t p_off[NLAYERS], nparams;  // canonical vector: weights at p_off, bias after them
};

// Validates and fills the shape from a descriptor; SV_OK or an error code.
sv_status net_shape(const sv_vae_desc *d, NetShape &ns);

// Spatial sizes: level 0 is the coarse map (ceil(H/f) x ceil(W/f)); level k+1
// halves level k (ceil); full resolution is H x W.
struct Levels {
    int H, W, h[4], w[4];
};
Levels net_levels(const NetShape &ns, int H, int W);
// 1 (default): an inference pass fuses the head and G3 where the widths allow
void net_set_latent_fusion(int on);

// Device tensors of one forward pass.  "saved" holds what the backward needs
// beyond the recomputed encoder; at inference it lives inside the workspace.
struct ActLayout {
    // workspace
    size_t E1, E2, E3, part, part_bytes, amax, ws_fwd;
    // saved (offsets within the saved region)
    size_t disp, img, ML, Z, G3, G2, G1, G0, saved;
};
ActLayout net_act_layout(const NetShape &ns, const Levels &lv, int B);

// Device bytes an inference pass uses: the workspace part plus the decoder
// maps and [mu | logvar] that live behind it when nothing is saved.
size_t net_infer_bytes(const NetShape &ns, const Levels &lv, int B);

// Extra workspace of the backward pass (after the forward's workspace part).
size_t net_bwd_workspace(const NetShape &ns, const Levels &lv, int B);

// INT8 passes: amax slots (AMAX_SUB words each) of the maps a layer reads
enum AmaxSlot { AM_E1 = 0, AM_E2, AM_E3, AM_ML, AM_G3, AM_G2, AM_G1, AM_G0, AM_X0, AM_NSLOTS };

// Tile configuration per layer (index into the conv kernel's table); the
// defaults may be replaced by the autotuner.
int net_default_cfg(const NetShape &ns, int layer, int M);
// Whether G0 carries the final layer's projection in its epilogue (inference
// in FP32 / BF16 / FP16, c1 <= 64), and the tile configuration it then runs:
// cfg's tile if it can hold every channel of G0 in each wave, else th4_tn32 /
// th4_tn64; never split.
bool net_projects(const NetShape &ns, bool train);
int net_g0_proj_cfg(const NetShape &ns, int cfg);
// The built-in choice for a layer, ignoring overrides and the autotune cache.
int net_heuristic_cfg(const NetShape &ns, int layer);
// Per-layer tile configuration of a forward pass of batch B at H x W: an
// explicit override, else the autotune cache entry for this shape, else the
// default.
void net_layer_cfgs(const NetShape &ns, int B, int H, int W, int *cfg);
// The reduction split a layer's configuration gives in a forward pass (1: none).
int net_layer_split(const NetShape &ns, int layer, int cfg, int B, int H, int W);
// The autotune cache entry for this network and image size with the nearest
// batch size; false if there is none.
bool tuned_lookup(const NetShape &ns, int B, int H, int W, int *cfg, int *dsplit);
void net_set_cfg_override(int dtype, int layer, int cfg);   // -1 restores the default
int net_get_cfg_override(int dtype, int layer);

// only >= 0: launch that network layer alone (for timing), nothing else;
// cfg_in (nullable, NLAYERS entries): the layers' configurations for this call
// in place of net_layer_cfgs (the autotuner passes its candidates this way)
sv_status net_forward(const NetShape &ns, const void *packed, const uint8_t *disp,
                      const uint8_t *img, int B, int H, int W, const float *eps, float *out,
                      float *ml_user, void *saved, void *ws, hipStream_t st, int only = -1,
                      const int *cfg_in = nullptr);

sv_status net_backward(const NetShape &ns, const void *packed, const void *saved, int B, int H,
                       int W, const float *eps, const float *dout, const float *dml_extra,
                       float kl_weight, float *grad, void *ws, hipStream_t st);

sv_status net_pack(const NetShape &ns, const float *params, void *packed, hipStream_t st);

}  // namespace sv
