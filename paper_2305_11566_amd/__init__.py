"""StereoVAE hot path on MI355X (gfx950): census + Hamming cost + winner-take-all
at reduced resolution, then the tiny VAE that upsamples and refines the coarse
map -- hand-written HIP kernels behind the C ABI of include/sv.h (libsv.so).

Python here only marshals arguments; see ``ops`` for the entry points.
"""
from ._lib import lib, header_symbols, SvError, SV_F32, SV_BF16, SV_F16, SV_I8, DTYPES  # noqa: F401
from .ops import (  # noqa: F401
    sv_census,
    sv_census_pair,
    sv_cost_wta,
    sv_sgm,
    sv_smp_median,
    sv_zncc_sgm,
    sv_zncc_cost,
    sv_set_cost_wta_split,
    sv_set_layer_cfg,
    sv_num_layer_cfgs,
    sv_set_latent_fusion,
    sv_conv_cfg_name,
    Refiner,
    vae_param_count,
    sv_profile_enable,
    sv_profile_repeat,
    sv_profile_read,
    PROFILE_STAGES,
    BatchPlan,
    PaperBatch,
    sv_autotune,
    sv_tile_config,
    sv_layer_cfgs,
    sv_loss,
    sv_adam_step,
    TableVAE,
    tvae_param_count,
    sv_tvae_loss,
    sv_tvae_set_layer_cfg,
    sv_tvae_num_layers,
    sv_tvae_set_deconv_form,
    sv_tvae_autotune,
    sv_tvae_layer_cfgs,
)
