"""ctypes binding of libsv.so (include/sv.h).

Argument marshalling only: every step of the path runs in the HIP library.
PyTorch supplies device memory and the current stream.  If the library is
not built, loading raises immediately -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsv.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "sv.h")

SV_F32, SV_BF16, SV_F16, SV_I8 = 0, 1, 2, 3
DTYPES = {"f32": SV_F32, "fp32": SV_F32, "bf16": SV_BF16, "f16": SV_F16, "fp16": SV_F16, "i8": SV_I8,
          "int8": SV_I8}

STATUS = {0: "SV_OK", -1: "SV_ERR_NULL", -2: "SV_ERR_SHAPE", -3: "SV_ERR_RANGE",
          -4: "SV_ERR_DTYPE", -5: "SV_ERR_WORKSPACE", -6: "SV_ERR_UNSUPPORTED", -7: "SV_ERR_HIP"}


class SvError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where} -> {STATUS.get(status, status)}" + (f" ({detail})" if detail else ""))


class VaeDesc(ctypes.Structure):
    _fields_ = [("c1", ctypes.c_int32), ("c2", ctypes.c_int32), ("c3", ctypes.c_int32),
                ("latent", ctypes.c_int32), ("factor", ctypes.c_int32), ("dtype", ctypes.c_int32)]


class PaperDesc(ctypes.Structure):
    _fields_ = [("matcher", ctypes.c_int32), ("factor", ctypes.c_int32), ("win_w", ctypes.c_int32),
                ("win_h", ctypes.c_int32), ("P1", ctypes.c_int32), ("P2", ctypes.c_int32),
                ("median", ctypes.c_int32), ("dtype", ctypes.c_int32)]


class Pair(ctypes.Structure):
    _fields_ = [("left", ctypes.c_void_p), ("right", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("disp_low", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("D", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_SZ = ctypes.c_size_t
_F = ctypes.c_float
_I64 = ctypes.c_int64
_DESC = ctypes.POINTER(VaeDesc)

_SIGS = {
    "sv_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "sv_last_error": (ctypes.c_char_p, []),
    "sv_census": (ctypes.c_int32, [_P, _I, _I, _I, _I, _I, _I, _I, _P, _P, _P]),
    "sv_census_pair": (ctypes.c_int32, [_P, _P, _I, _I, _I, _I, _I, _I, _I, _P, _P, _P, _P]),
    "sv_cost_wta": (ctypes.c_int32, [_P, _P, _I, _I, _I, _I, _I, _P, _P]),
    "sv_set_cost_wta_split": (ctypes.c_int32, [_I]),
    "sv_sgm_workspace_bytes": (ctypes.c_size_t, [_I, _I, _I, _I]),
    "sv_sgm": (ctypes.c_int32, [_P, _P, _I, _I, _I, _I, _I, _I, _I, _P, _P, ctypes.c_size_t, _P]),
    "sv_smp_workspace_bytes": (ctypes.c_size_t, [_I, _I, _I]),
    "sv_zncc_sgm": (ctypes.c_int32, [_P, _P, _I, _I, _I, _I, _I, _I, _I, _I, _P, _P, ctypes.c_size_t, _P]),
    "sv_zncc_cost": (ctypes.c_int32, [_P, _P, _I, _I, _I, _I, _I, _I, _P, _P]),
    "sv_smp_median": (ctypes.c_int32, [_P, _I, _I, _I, _I, _P, _P, ctypes.c_size_t, _P]),
    "sv_vae_param_count": (_I64, [_DESC]),
    "sv_vae_packed_bytes": (_SZ, [_DESC]),
    "sv_vae_pack_weights": (ctypes.c_int32, [_DESC, _P, _P, _P]),
    "sv_vae_workspace_bytes": (_SZ, [_DESC, _I, _I, _I]),
    "sv_vae_saved_bytes": (_SZ, [_DESC, _I, _I, _I]),
    "sv_vae_forward": (ctypes.c_int32, [_DESC, _P, _P, _P, _I, _I, _I, _P, _P, _P, _P, _P, _SZ, _P]),
    "sv_vae_forward_static": (ctypes.c_int32, [_DESC, _P, _P, _P, _I, _I, _I, _P, _P, _P]),
    "sv_vae_backward": (ctypes.c_int32, [_DESC, _P, _P, _I, _I, _I, _P, _P, _P, _F, _P, _P, _SZ, _P]),
    "sv_loss": (ctypes.c_int32, [_P, _P, _I64, _P, _I64, _I, _F, _P, _P, _P, _SZ, _P]),
    "sv_loss_workspace_bytes": (_SZ, []),
    "sv_adam_step": (ctypes.c_int32, [_P, _P, _P, _P, _I64, _I, _F, _F, _F, _F, _P]),
    "sv_set_layer_cfg": (ctypes.c_int32, [_I, _I]),
    "sv_num_layer_cfgs": (_I, []),
    "sv_set_latent_fusion": (ctypes.c_int32, [_I]),
    "sv_batch_plan_create": (ctypes.c_int32, [_DESC, _I, _I, _I, _I, _I, _I, ctypes.POINTER(_P)]),
    "sv_batch_plan_destroy": (ctypes.c_int32, [_P]),
    "sv_stereo_batch": (ctypes.c_int32, [_P, ctypes.POINTER(Pair), _I, _P, _P]),
    "sv_autotune": (ctypes.c_int32, [_DESC, _I, _I, _I, _I, _I, _I]),
    "sv_tile_config": (ctypes.c_int32, [_I, ctypes.c_char_p, _I]),
    "sv_paper_batch_workspace_bytes": (ctypes.c_size_t, [_P, _I, _I, _I]),
    "sv_paper_batch": (ctypes.c_int32, [_P, _P, _I, _P, _P, ctypes.c_size_t, _P]),
    "sv_profile_enable": (ctypes.c_int32, [_I]),
    "sv_profile_repeat": (ctypes.c_int32, [_I]),
    "sv_layer_cfgs": (ctypes.c_int32, [_DESC, _I, _I, _I, ctypes.POINTER(ctypes.c_int)]),
    "sv_conv_cfg_name": (ctypes.c_char_p, [_I]),
    "sv_profile_read": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int)]),
    "sv_tvae_param_count": (_I64, []),
    "sv_tvae_packed_bytes": (_SZ, [_I]),
    "sv_tvae_pack_weights": (ctypes.c_int32, [_I, _P, _P, _P]),
    "sv_tvae_workspace_bytes": (_SZ, [_I, _I, _I, _I, _I]),
    "sv_tvae_forward": (ctypes.c_int32, [_I, _I, _P, _P, _P, _I, _I, _I, _P, _P, _P, _P, _SZ, _P]),
    "sv_tvae_loss_workspace_bytes": (_SZ, []),
    "sv_tvae_loss": (ctypes.c_int32, [_P, _P, _P, _P, _I64, _P, _I64, _P, _P, _P, _P, _SZ, _P]),
    "sv_tvae_set_layer_cfg": (ctypes.c_int32, [_I, _I]),
    "sv_tvae_num_layers": (_I, []),
    "sv_tvae_set_deconv_form": (ctypes.c_int32, [_I]),
    "sv_tvae_autotune": (ctypes.c_int32, [_I, _I, _I, _I, _I]),
    "sv_tvae_backward_workspace_bytes": (_SZ, [_I, _I, _I, _I, _I]),
    "sv_tvae_backward": (ctypes.c_int32, [_I, _I, _P, _P, _P, _I, _I, _I, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "sv_tvae_layer_cfgs": (ctypes.c_int32, [_I, _I, _I, _I, _I, ctypes.POINTER(ctypes.c_int)]),
}


def lib():
    """Loads libsv.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950). There is no CPU fallback.")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(l, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def header_symbols() -> list[str]:
    """Function names declared in include/sv.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z0-9_]+)\s*\(", txt)))


def check(status: int, where: str) -> None:
    if status != 0:
        detail = lib().sv_last_error().decode() if status == -7 else ""
        raise SvError(status, where, detail)


def ptr(t) -> ctypes.c_void_p | None:
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def stream_ptr(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_desc(c1: int, c2: int, c3: int, latent: int, factor: int, dtype) -> VaeDesc:
    dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    return VaeDesc(c1, c2, c3, latent, factor, dt)
