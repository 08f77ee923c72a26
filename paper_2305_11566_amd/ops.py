"""Python entry points with the C ABI's names, over torch tensors on the GPU.

Each function only allocates outputs (torch), marshals pointers and calls
libsv.so on the current stream.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import (SV_F32, check, lib, make_desc, ptr, stream_ptr, VaeDesc, DTYPES)


def _cdiv(a, b):
    return -(-a // b)


def _need(t, dtype, name, shape=None, device=None):
    """Checks a tensor handed to the library: a contiguous GPU tensor of this
    dtype and, when given, this shape and device.  The C ABI sees only a
    pointer, so a buffer of the wrong size must be refused here, before any
    call (a kernel would read or write past it)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if device is not None and not _same_device(t.device, device):
        raise ValueError(f"{name} is on {t.device}, expected {device}")


def _same_device(a, b):
    """torch.device("cuda") names the current device: compare indices."""
    a, b = torch.device(a), torch.device(b)
    if a.type != b.type:
        return False
    ia = a.index if a.index is not None else torch.cuda.current_device()
    ib = b.index if b.index is not None else torch.cuda.current_device()
    return ia == ib


def _need_numel(t, dtype, name, n, device=None):
    """As _need, for a flat buffer of at least n elements."""
    _need(t, dtype, name, device=device)
    if t.numel() < n:
        raise ValueError(f"{name} must hold at least {n} elements, got {t.numel()}")


# ---------------------------------------------------------------- matching

def sv_census(img: torch.Tensor, factor: int, win_w: int, win_h: int, want_low: bool = True,
              out: tuple | None = None):
    """uint8 [B, H, W] -> (census int64-bits [B, h, w], reduced image uint8 [B, h, w] or None);
    `out` = (census, reduced image) preallocated."""
    _need(img, torch.uint8, "img")
    if img.dim() == 2:
        img = img[None]
    B, H, W = img.shape
    h, w = _cdiv(H, factor), _cdiv(W, factor)
    if out is not None:
        cen, low = out
        _need(cen, torch.int64, "census out", (B, h, w), img.device)
        if low is not None:
            _need(low, torch.uint8, "reduced image out", (B, h, w), img.device)
    else:
        cen = torch.empty((B, h, w), dtype=torch.int64, device=img.device)
        low = torch.empty((B, h, w), dtype=torch.uint8, device=img.device) if want_low else None
    check(lib().sv_census(ptr(img), B, H, W, W, factor, win_w, win_h, ptr(low), ptr(cen),
                          stream_ptr()), "sv_census")
    return cen, low


def sv_census_pair(left: torch.Tensor, right: torch.Tensor, factor: int, win_w: int, win_h: int,
                   out=None):
    """Both views in one launch -> (census L, census R, reduced left image).
    out: optional preallocated (census L, census R, reduced left)."""
    _need(left, torch.uint8, "left")
    _need(right, torch.uint8, "right")
    if left.dim() == 2:
        left, right = left[None], right[None]
    if left.shape != right.shape:
        raise ValueError("left and right must have the same shape")
    B, H, W = left.shape
    h, w = _cdiv(H, factor), _cdiv(W, factor)
    if out is None:
        cl = torch.empty((B, h, w), dtype=torch.int64, device=left.device)
        cr = torch.empty_like(cl)
        low = torch.empty((B, h, w), dtype=torch.uint8, device=left.device)
    else:
        cl, cr, low = out
        _need(cl, torch.int64, "census L out", (B, h, w), left.device)
        _need(cr, torch.int64, "census R out", (B, h, w), left.device)
        _need(low, torch.uint8, "reduced image out", (B, h, w), left.device)
    check(lib().sv_census_pair(ptr(left), ptr(right), B, H, W, W, factor, win_w, win_h, ptr(low),
                               ptr(cl), ptr(cr), stream_ptr()), "sv_census_pair")
    return cl, cr, low


def sv_cost_wta(cen_l: torch.Tensor, cen_r: torch.Tensor, D: int, nbits: int,
                out: torch.Tensor | None = None):
    """Census maps (int64 bits) [B, h, w] -> WTA disparity uint8 [B, h, w]."""
    _need(cen_l, torch.int64, "cen_l")
    _need(cen_r, torch.int64, "cen_r")
    if cen_l.shape != cen_r.shape:
        raise ValueError("census maps differ in shape")
    B, h, w = cen_l.shape
    if out is None:
        out = torch.empty((B, h, w), dtype=torch.uint8, device=cen_l.device)
    _need(out, torch.uint8, "out", (B, h, w), cen_l.device)
    check(lib().sv_cost_wta(ptr(cen_l), ptr(cen_r), B, h, w, D, nbits, ptr(out), stream_ptr()),
          "sv_cost_wta")
    return out


def sv_sgm(cen_l: torch.Tensor, cen_r: torch.Tensor, D: int, nbits: int, P1: int, P2: int,
           out: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """Census maps (int64 bits) [B, h, w] -> semi-global matching disparity uint8
    [B, h, w] (four axis paths, Eqs. (4)-(6)).  The path-cost volumes live in
    `workspace` (uint8, at least sv_sgm_workspace_bytes) when given."""
    _need(cen_l, torch.int64, "cen_l")
    _need(cen_r, torch.int64, "cen_r")
    if cen_l.shape != cen_r.shape:
        raise ValueError("census maps differ in shape")
    B, h, w = cen_l.shape
    need = lib().sv_sgm_workspace_bytes(B, h, w, D)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=cen_l.device)
    if out is None:
        out = torch.empty((B, h, w), dtype=torch.uint8, device=cen_l.device)
    _need(out, torch.uint8, "out", (B, h, w), cen_l.device)
    _need_numel(workspace, torch.uint8, "workspace", need, cen_l.device)
    check(lib().sv_sgm(ptr(cen_l), ptr(cen_r), B, h, w, D, nbits, P1, P2, ptr(out), ptr(workspace),
                       workspace.numel(), stream_ptr()), "sv_sgm")
    return out


def sv_zncc_sgm(low_l: torch.Tensor, low_r: torch.Tensor, D: int, win_w: int, win_h: int, P1: int,
                P2: int, out: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """Reduced images uint8 [B, h, w] -> ZNCC + SGM disparity uint8 [B, h, w]."""
    _need(low_l, torch.uint8, "low_l")
    _need(low_r, torch.uint8, "low_r")
    if low_l.shape != low_r.shape:
        raise ValueError("images differ in shape")
    B, h, w = low_l.shape
    if workspace is None:
        workspace = torch.empty(max(lib().sv_sgm_workspace_bytes(B, h, w, D), 1), dtype=torch.uint8,
                                device=low_l.device)
    if out is None:
        out = torch.empty((B, h, w), dtype=torch.uint8, device=low_l.device)
    _need(out, torch.uint8, "out", (B, h, w), low_l.device)
    _need_numel(workspace, torch.uint8, "workspace", lib().sv_sgm_workspace_bytes(B, h, w, D), low_l.device)
    check(lib().sv_zncc_sgm(ptr(low_l), ptr(low_r), B, h, w, D, win_w, win_h, P1, P2, ptr(out),
                            ptr(workspace), workspace.numel(), stream_ptr()), "sv_zncc_sgm")
    return out


def sv_zncc_cost(low_l: torch.Tensor, low_r: torch.Tensor, D: int, win_w: int, win_h: int):
    """Reduced images uint8 [B, h, w] -> integer ZNCC cost uint8 [B, h, w, D]."""
    _need(low_l, torch.uint8, "low_l")
    if low_l.dim() != 3:
        raise ValueError("low_l must be [B, h, w]")
    B, h, w = low_l.shape
    _need(low_r, torch.uint8, "low_r", (B, h, w), low_l.device)
    out = torch.empty((B, h, w, D), dtype=torch.uint8, device=low_l.device)
    check(lib().sv_zncc_cost(ptr(low_l), ptr(low_r), B, h, w, D, win_w, win_h, ptr(out), stream_ptr()),
          "sv_zncc_cost")
    return out


def sv_smp_median(disp: torch.Tensor, D: int, out: torch.Tensor | None = None,
                  workspace: torch.Tensor | None = None):
    """Single matching phase (Eq. (7)) with nearest-valid filling, then a 3 x 3
    median: uint8 [B, h, w] -> uint8 [B, h, w]."""
    _need(disp, torch.uint8, "disp")
    B, h, w = disp.shape
    if workspace is None:
        workspace = torch.empty(max(lib().sv_smp_workspace_bytes(B, h, w), 1), dtype=torch.uint8,
                                device=disp.device)
    if out is None:
        out = torch.empty_like(disp)
    _need(out, torch.uint8, "out", (B, h, w), disp.device)
    _need_numel(workspace, torch.uint8, "workspace", lib().sv_smp_workspace_bytes(B, h, w), disp.device)
    check(lib().sv_smp_median(ptr(disp), B, h, w, D, ptr(out), ptr(workspace), workspace.numel(),
                              stream_ptr()), "sv_smp_median")
    return out


def sv_set_cost_wta_split(dsplit: int):
    check(lib().sv_set_cost_wta_split(dsplit), "sv_set_cost_wta_split")


def sv_set_layer_cfg(layer: int, cfg: int):
    check(lib().sv_set_layer_cfg(layer, cfg), "sv_set_layer_cfg")


def sv_num_layer_cfgs() -> int:
    return lib().sv_num_layer_cfgs()


def sv_set_latent_fusion(on: bool):
    """Inference passes run the latent head and G3 as one kernel (default) or
    as two launches; both give the same bits."""
    check(lib().sv_set_latent_fusion(1 if on else 0), "sv_set_latent_fusion")


def sv_conv_cfg_name(cfg: int) -> str:
    """Name of a layer configuration: the tile shape, plus "_s<k>" for a
    k-way split of the channel reduction."""
    return lib().sv_conv_cfg_name(cfg).decode()


# ----------------------------------------------------------------- network

def _aligned_bytes(n: int, device) -> torch.Tensor:
    """A uint8 buffer of at least n bytes whose start is 256-byte aligned."""
    buf = torch.empty(max(n, 1) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + max(n, 1)]


class Refiner:
    """Holds a network descriptor, packed weights and a workspace sized for
    the last shape; forwards to sv_vae_forward / sv_vae_backward."""

    def __init__(self, c1, c2, c3, latent, factor, dtype="f32", device="cuda"):
        self.desc = make_desc(c1, c2, c3, latent, factor, dtype)
        self.device = torch.device(device)
        self.nparams = int(lib().sv_vae_param_count(ctypes.byref(self.desc)))
        check(0 if self.nparams > 0 else self.nparams, "sv_vae_param_count")
        self.packed = _aligned_bytes(lib().sv_vae_packed_bytes(ctypes.byref(self.desc)), self.device)
        self._ws = None
        self._ws_key = None

    @property
    def dtype_code(self):
        return self.desc.dtype

    def pack(self, params: torch.Tensor):
        """params: FP32 canonical vector [nparams] on the device."""
        _need(params, torch.float32, "params")
        if params.numel() != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {params.numel()}")
        check(lib().sv_vae_pack_weights(ctypes.byref(self.desc), ptr(params), ptr(self.packed),
                                        stream_ptr()), "sv_vae_pack_weights")

    def workspace(self, B, H, W):
        key = (B, H, W)
        if self._ws_key != key:
            n = lib().sv_vae_workspace_bytes(ctypes.byref(self.desc), B, H, W)
            if n == 0:
                raise ValueError(f"invalid shape {key}")
            self._ws = _aligned_bytes(n, self.device)
            self._ws_key = key
        return self._ws

    def saved_buffer(self, B, H, W):
        return _aligned_bytes(lib().sv_vae_saved_bytes(ctypes.byref(self.desc), B, H, W), self.device)

    def latent_shape(self, B, H, W):
        f = self.desc.factor
        h, w = _cdiv(H, f), _cdiv(W, f)
        for _ in range(3):
            h, w = _cdiv(h, 2), _cdiv(w, 2)
        return (B, h, w, self.desc.latent)

    def forward(self, disp_low, img_low, H, W, eps=None, saved=None, out=None, mu_logvar=None):
        """-> (out [B, H, W] full-res px, mu_logvar [B, h3, w3, 2L])."""
        if disp_low.dim() != 3:
            raise ValueError("disp_low must be [B, h, w]")
        B = disp_low.shape[0]
        f = self.desc.factor
        low = (B, _cdiv(H, f), _cdiv(W, f))
        dev = self.device
        _need(disp_low, torch.uint8, "disp_low", low, dev)
        _need(img_low, torch.uint8, "img_low", low, dev)
        s = self.latent_shape(B, H, W)
        if out is None:
            out = torch.empty((B, H, W), dtype=torch.float32, device=dev)
        if mu_logvar is None:
            mu_logvar = torch.empty(s[:3] + (2 * s[3],), dtype=torch.float32, device=dev)
        _need(out, torch.float32, "out", (B, H, W), dev)
        _need(mu_logvar, torch.float32, "mu_logvar", s[:3] + (2 * s[3],), dev)
        if eps is not None:
            _need(eps, torch.float32, "eps", s, dev)
            if saved is None:
                raise ValueError("training forward needs a saved buffer")
        if saved is not None:
            _need_numel(saved, torch.uint8, "saved",
                        lib().sv_vae_saved_bytes(ctypes.byref(self.desc), B, H, W), dev)
        ws = self.workspace(B, H, W)
        check(lib().sv_vae_forward(ctypes.byref(self.desc), ptr(self.packed), ptr(disp_low),
                                   ptr(img_low), B, H, W, ptr(eps), ptr(out), ptr(mu_logvar),
                                   ptr(saved), ptr(ws), ws.numel(), stream_ptr()), "sv_vae_forward")
        return out, mu_logvar

    def forward_static(self, disp_low, img_low, H, W, out=None, mu_logvar=None):
        """Inference through sv_vae_forward_static (the library's own fixed
        scratch, no workspace) -> (out [B, H, W], mu_logvar [B, h3, w3, 2L])."""
        if disp_low.dim() != 3:
            raise ValueError("disp_low must be [B, h, w]")
        B = disp_low.shape[0]
        f = self.desc.factor
        low = (B, _cdiv(H, f), _cdiv(W, f))
        dev = self.device
        _need(disp_low, torch.uint8, "disp_low", low, dev)
        _need(img_low, torch.uint8, "img_low", low, dev)
        s = self.latent_shape(B, H, W)
        if out is None:
            out = torch.empty((B, H, W), dtype=torch.float32, device=dev)
        if mu_logvar is None:
            mu_logvar = torch.empty(s[:3] + (2 * s[3],), dtype=torch.float32, device=dev)
        _need(out, torch.float32, "out", (B, H, W), dev)
        _need(mu_logvar, torch.float32, "mu_logvar", s[:3] + (2 * s[3],), dev)
        check(lib().sv_vae_forward_static(ctypes.byref(self.desc), ptr(self.packed), ptr(disp_low),
                                          ptr(img_low), B, H, W, ptr(out), ptr(mu_logvar), stream_ptr()),
              "sv_vae_forward_static")
        return out, mu_logvar

    def backward(self, saved, B, H, W, eps, dout, kl_weight, grad=None, dmu_logvar=None):
        """Gradient of sum(dout * out) + kl_weight * KL (+ sum(dmu_logvar * mu_logvar))."""
        dev = self.device
        s = self.latent_shape(B, H, W)
        _need(dout, torch.float32, "dout", (B, H, W), dev)
        _need_numel(saved, torch.uint8, "saved", lib().sv_vae_saved_bytes(ctypes.byref(self.desc), B, H, W),
                    dev)
        if eps is not None:
            _need(eps, torch.float32, "eps", s, dev)
        if dmu_logvar is not None:
            _need(dmu_logvar, torch.float32, "dmu_logvar", s[:3] + (2 * s[3],), dev)
        if grad is None:
            grad = torch.empty(self.nparams, dtype=torch.float32, device=dev)
        _need(grad, torch.float32, "grad", (self.nparams,), dev)
        ws = self.workspace(B, H, W)
        check(lib().sv_vae_backward(ctypes.byref(self.desc), ptr(self.packed), ptr(saved), B, H, W,
                                    ptr(eps), ptr(dout), ptr(dmu_logvar), ctypes.c_float(kl_weight),
                                    ptr(grad), ptr(ws), ws.numel(), stream_ptr()), "sv_vae_backward")
        return grad


def sv_profile_enable(max_calls: int):
    check(lib().sv_profile_enable(max_calls), "sv_profile_enable")


def sv_profile_repeat(repeat: int):
    check(lib().sv_profile_repeat(repeat), "sv_profile_repeat")


PROFILE_STAGES = ("census", "cost_wta", "E1", "E2", "E3", "HEAD", "reparam", "G3", "G2", "G1",
                  "G0", "final_proj", "final_gather", "split_sum")


def sv_profile_read():
    """-> {stage: (summed ms, launches)}; synchronises on the recorded events."""
    n = len(PROFILE_STAGES)
    ms = (ctypes.c_float * n)()
    cnt = (ctypes.c_int * n)()
    check(lib().sv_profile_read(ms, cnt), "sv_profile_read")
    return {PROFILE_STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}


def vae_param_count(c1, c2, c3, latent, factor=2, dtype="f32") -> int:
    d = make_desc(c1, c2, c3, latent, factor, dtype)
    return int(lib().sv_vae_param_count(ctypes.byref(d)))


# ----------------------------------------------------------------- training

def sv_loss(out, gt, mu_logvar, latent, kl_weight, loss_out=None, dout=None, workspace=None):
    """-> (loss[3] = {total, data, KL} on the device, dout).  mu_logvar may be None."""
    _need(out, torch.float32, "out")
    dev = out.device
    _need(gt, torch.float32, "gt", out.shape, dev)
    if loss_out is None:
        loss_out = torch.empty(3, dtype=torch.float32, device=dev)
    if dout is None:
        dout = torch.empty_like(out)
    if workspace is None:
        workspace = torch.empty(lib().sv_loss_workspace_bytes(), dtype=torch.uint8, device=dev)
    _need(loss_out, torch.float32, "loss_out", (3,), dev)
    _need(dout, torch.float32, "dout", out.shape, dev)
    _need_numel(workspace, torch.uint8, "workspace", lib().sv_loss_workspace_bytes(), dev)
    if mu_logvar is not None:
        _need(mu_logvar, torch.float32, "mu_logvar", device=dev)
        if mu_logvar.shape[-1] != 2 * latent:
            raise ValueError(f"mu_logvar rows must hold 2 * latent = {2 * latent} values")
    n_lat = 0 if mu_logvar is None else mu_logvar.numel() // (2 * latent)
    check(lib().sv_loss(ptr(out), ptr(gt), out.numel(), ptr(mu_logvar), n_lat, latent,
                        ctypes.c_float(kl_weight), ptr(loss_out), ptr(dout), ptr(workspace),
                        workspace.numel(), stream_ptr()), "sv_loss")
    return loss_out, dout


def sv_adam_step(w, g, m, v, step, lr=5e-4, beta1=0.99, beta2=0.999, eps=1e-8):
    for t, n in ((w, "w"), (g, "g"), (m, "m"), (v, "v")):
        _need(t, torch.float32, n, w.shape, w.device)
    check(lib().sv_adam_step(ptr(w), ptr(g), ptr(m), ptr(v), w.numel(), step, ctypes.c_float(lr),
                             ctypes.c_float(beta1), ctypes.c_float(beta2), ctypes.c_float(eps),
                             stream_ptr()), "sv_adam_step")


# ------------------------------------------------------------ batches of pairs

class BatchPlan:
    """sv_batch_plan: uneven pairs through the whole path in one graph replay."""

    def __init__(self, c1, c2, c3, latent, factor, dtype, max_n, max_H, max_W, max_D, win_w, win_h):
        from ._lib import Pair  # noqa: F401
        self.desc = make_desc(c1, c2, c3, latent, factor, dtype)
        self.factor = factor
        self._plan = ctypes.c_void_p()
        check(lib().sv_batch_plan_create(ctypes.byref(self.desc), max_n, max_H, max_W, max_D, win_w,
                                         win_h, ctypes.byref(self._plan)), "sv_batch_plan_create")

    def run(self, pairs, packed, outs=None, disp_outs=None):
        """pairs: list of (left uint8 [H,W], right uint8 [H,W], D).  Returns the
        refined maps (float32 [H,W] each, full-res px)."""
        from ._lib import Pair
        n = len(pairs)
        arr = (Pair * n)()
        if outs is None:
            outs = [torch.empty(l.shape, dtype=torch.float32, device=l.device) for l, _, _ in pairs]
        if len(outs) != n or (disp_outs is not None and len(disp_outs) != n):
            raise ValueError("one output (and coarse map) per pair")
        for i, (l, r, D) in enumerate(pairs):
            _need(l, torch.uint8, "left")
            if l.dim() != 2:
                raise ValueError("left must be [H, W]")
            H, W = l.shape
            _need(r, torch.uint8, "right", (H, W), l.device)
            _need(outs[i], torch.float32, "out", (H, W), l.device)
            dl = disp_outs[i] if disp_outs is not None else None
            if dl is not None:
                _need(dl, torch.uint8, "disp_out", (_cdiv(H, self.factor), _cdiv(W, self.factor)), l.device)
            arr[i] = Pair(l.data_ptr(), r.data_ptr(), outs[i].data_ptr(),
                          dl.data_ptr() if dl is not None else None, H, W, D)
        check(lib().sv_stereo_batch(self._plan, arr, n, ptr(packed), stream_ptr()), "sv_stereo_batch")
        return outs

    def close(self):
        if self._plan:
            lib().sv_batch_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PaperBatch:
    """sv_paper_batch: the paper's whole system (reduction, ZNCC + SGM or census
    + SGM, single matching phase + median, Table I network) on pairs of uneven
    sizes, one launch sequence per call on the current stream (capturable in
    one graph); the workspace is sized for the largest pair."""

    MATCHERS = {"zncc": 0, "census": 1}

    def __init__(self, matcher, factor, win_w, win_h, P1, P2, dtype="f32", median=True, max_H=384, max_W=1280,
                 max_D=80, device="cuda"):
        from ._lib import PaperDesc
        if matcher not in self.MATCHERS or dtype not in DTYPES:
            raise ValueError(f"matcher in {list(self.MATCHERS)}, dtype in {list(DTYPES)}")
        self.desc = PaperDesc(self.MATCHERS[matcher], factor, win_w, win_h, P1, P2, 1 if median else 0,
                              DTYPES[dtype])
        self.factor = factor
        n = lib().sv_paper_batch_workspace_bytes(ctypes.byref(self.desc), max_H, max_W, max_D)
        if n == 0:
            raise ValueError("invalid matcher settings or sizes")
        self.workspace = _aligned_bytes(n, torch.device(device))

    def run(self, pairs, packed, outs=None, disp_outs=None):
        """pairs: list of (left uint8 [H,W], right uint8 [H,W], D); packed: the
        Table I network's packed weights (TableVAE.packed).  Returns the
        network's outputs (float32 [H,W] each, full-res px)."""
        from ._lib import Pair
        n = len(pairs)
        arr = (Pair * n)()
        if outs is None:
            outs = [torch.empty(l.shape, dtype=torch.float32, device=l.device) for l, _, _ in pairs]
        if len(outs) != n or (disp_outs is not None and len(disp_outs) != n):
            raise ValueError("one output (and coarse map) per pair")
        for i, (l, r, D) in enumerate(pairs):
            _need(l, torch.uint8, "left")
            if l.dim() != 2:
                raise ValueError("left must be [H, W]")
            H, W = l.shape
            _need(r, torch.uint8, "right", (H, W), l.device)
            _need(outs[i], torch.float32, "out", (H, W), l.device)
            dl = disp_outs[i] if disp_outs is not None else None
            if dl is not None:
                _need(dl, torch.uint8, "disp_out", (_cdiv(H, self.factor), _cdiv(W, self.factor)), l.device)
            arr[i] = Pair(l.data_ptr(), r.data_ptr(), outs[i].data_ptr(),
                          dl.data_ptr() if dl is not None else None, H, W, D)
        check(lib().sv_paper_batch(ctypes.byref(self.desc), arr, n, ptr(packed), ptr(self.workspace),
                                   self.workspace.numel(), stream_ptr()), "sv_paper_batch")
        return outs


def sv_autotune(c1, c2, c3, latent, factor, dtype, B, H, W, D, win_w, win_h):
    d = make_desc(c1, c2, c3, latent, factor, dtype)
    check(lib().sv_autotune(ctypes.byref(d), B, H, W, D, win_w, win_h), "sv_autotune")


def sv_layer_cfgs(c1, c2, c3, latent, factor, dtype, B, H, W):
    """Names of the tile configurations the 9 layers use for this shape."""
    d = make_desc(c1, c2, c3, latent, factor, dtype)
    out = (ctypes.c_int * 9)()
    check(lib().sv_layer_cfgs(ctypes.byref(d), B, H, W, out), "sv_layer_cfgs")
    return [lib().sv_conv_cfg_name(out[i]).decode() for i in range(9)]


def sv_tile_config(stage: int) -> str:
    buf = ctypes.create_string_buffer(128)
    check(lib().sv_tile_config(stage, buf, 128), "sv_tile_config")
    return buf.value.decode()

# ---------------------------------------------------------- Table I network

def tvae_param_count() -> int:
    return int(lib().sv_tvae_param_count())


def sv_tvae_set_layer_cfg(layer: int, cfg: int):
    check(lib().sv_tvae_set_layer_cfg(layer, cfg), "sv_tvae_set_layer_cfg")


def sv_tvae_set_deconv_form(form: int):
    check(lib().sv_tvae_set_deconv_form(form), "sv_tvae_set_deconv_form")


def sv_tvae_num_layers() -> int:
    return int(lib().sv_tvae_num_layers())


def sv_tvae_autotune(dtype: str, factor: int, B: int, H: int, W: int):
    check(lib().sv_tvae_autotune(DTYPES[dtype], factor, B, H, W), "sv_tvae_autotune")


def sv_tvae_layer_cfgs(dtype: str, factor: int, B: int, H: int, W: int) -> list[str]:
    n = sv_tvae_num_layers()
    arr = (ctypes.c_int * n)()
    check(lib().sv_tvae_layer_cfgs(DTYPES[dtype], factor, B, H, W, arr), "sv_tvae_layer_cfgs")
    return [lib().sv_conv_cfg_name(c).decode() for c in arr]


class TableVAE:
    """The Table I network: packed weights and a workspace sized for the last
    shape; forwards to sv_tvae_forward."""

    def __init__(self, factor, dtype="f32", device="cuda"):
        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {sorted(DTYPES)}")
        self.dtype_code = DTYPES[dtype]
        self.factor = factor
        self.device = torch.device(device)
        self.nparams = tvae_param_count()
        self.packed = _aligned_bytes(lib().sv_tvae_packed_bytes(self.dtype_code), self.device)
        self._ws = None
        self._ws_key = None

    def pack(self, params: torch.Tensor):
        """params: FP32 canonical vector [nparams] on the device."""
        _need(params, torch.float32, "params")
        if params.numel() != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {params.numel()}")
        check(lib().sv_tvae_pack_weights(self.dtype_code, ptr(params), ptr(self.packed), stream_ptr()),
              "sv_tvae_pack_weights")

    def workspace(self, B, H, W):
        key = (B, H, W)
        if self._ws_key != key:
            n = lib().sv_tvae_workspace_bytes(self.dtype_code, self.factor, B, H, W)
            if n == 0:
                raise ValueError(f"invalid shape {key}")
            self._ws = _aligned_bytes(n, self.device)
            self._ws_key = key
        return self._ws

    def latent_shape(self, B, H, W):
        h, w = _cdiv(H, self.factor), _cdiv(W, self.factor)
        for _ in range(2):
            h, w = _cdiv(h, 2), _cdiv(w, 2)
        return (B, h, w)

    def forward(self, disp_low, img_low, H, W, eps=None, out=None, mu_sigma=None):
        """-> (out [B, H, W] full-res px, mu_sigma [B, h3, w3, 2])."""
        if disp_low.dim() != 3:
            raise ValueError("disp_low must be [B, h, w]")
        B = disp_low.shape[0]
        dev = self.device
        low = (B, _cdiv(H, self.factor), _cdiv(W, self.factor))
        _need(disp_low, torch.uint8, "disp_low", low, dev)
        _need(img_low, torch.uint8, "img_low", low, dev)
        if out is None:
            out = torch.empty((B, H, W), dtype=torch.float32, device=dev)
        if mu_sigma is None:
            mu_sigma = torch.empty(self.latent_shape(B, H, W) + (2,), dtype=torch.float32, device=dev)
        _need(out, torch.float32, "out", (B, H, W), dev)
        _need(mu_sigma, torch.float32, "mu_sigma", self.latent_shape(B, H, W) + (2,), dev)
        if eps is not None:
            _need(eps, torch.float32, "eps", self.latent_shape(B, H, W), dev)
        ws = self.workspace(B, H, W)
        check(lib().sv_tvae_forward(self.dtype_code, self.factor, ptr(self.packed), ptr(disp_low),
                                    ptr(img_low), B, H, W, ptr(eps), ptr(out), ptr(mu_sigma), ptr(ws),
                                    ws.numel(), stream_ptr()), "sv_tvae_forward")
        return out, mu_sigma

    def backward(self, disp_low, img_low, H, W, dout, eps=None, dmu_sigma=None, grad=None):
        """Gradient of sum(dout * out) + sum(dmu_sigma * mu_sigma) after forward() on the
        same inputs (its workspace holds the activations)."""
        B = disp_low.shape[0]
        dev = self.device
        low = (B, _cdiv(H, self.factor), _cdiv(W, self.factor))
        _need(disp_low, torch.uint8, "disp_low", low, dev)
        _need(img_low, torch.uint8, "img_low", low, dev)
        _need(dout, torch.float32, "dout", (B, H, W), dev)
        if eps is not None:
            _need(eps, torch.float32, "eps", self.latent_shape(B, H, W), dev)
        if dmu_sigma is not None:
            _need(dmu_sigma, torch.float32, "dmu_sigma", self.latent_shape(B, H, W) + (2,), dev)
        if self._ws_key != (B, H, W):
            raise ValueError("backward() needs the forward pass of the same shape just before")
        if grad is None:
            grad = torch.empty(self.nparams, dtype=torch.float32, device=dev)
        _need(grad, torch.float32, "grad", (self.nparams,), dev)
        key = ("bwd", B, H, W)
        if getattr(self, "_bws_key", None) != key:
            n = lib().sv_tvae_backward_workspace_bytes(self.dtype_code, self.factor, B, H, W)
            self._bws = _aligned_bytes(n, self.device)
            self._bws_key = key
        check(lib().sv_tvae_backward(self.dtype_code, self.factor, ptr(self.packed), ptr(disp_low),
                                     ptr(img_low), B, H, W, ptr(eps), ptr(self._ws), ptr(dout),
                                     ptr(dmu_sigma), ptr(grad), ptr(self._bws), self._bws.numel(),
                                     stream_ptr()), "sv_tvae_backward")
        return grad


def sv_tvae_loss(out, gt, noc, occ, mu_sigma, want_grad=True):
    """Eqs. (9)-(11) -> (loss [3] = total, Loss_1, Loss_2; dout or None; dmu_sigma or None)."""
    _need(out, torch.float32, "out")
    dev = out.device
    _need(gt, torch.float32, "gt", out.shape, dev)
    _need(noc, torch.uint8, "noc", out.shape, dev)
    _need(occ, torch.uint8, "occ", out.shape, dev)
    _need(mu_sigma, torch.float32, "mu_sigma", device=dev)
    if mu_sigma.shape[-1] != 2:
        raise ValueError("mu_sigma must be [..., 2]")
    loss = torch.empty(3, dtype=torch.float32, device=out.device)
    dout = torch.empty_like(out) if want_grad else None
    dml = torch.empty_like(mu_sigma) if want_grad else None
    nb = lib().sv_tvae_loss_workspace_bytes()
    ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device=out.device)
    check(lib().sv_tvae_loss(ptr(out), ptr(gt), ptr(noc), ptr(occ), out.numel(), ptr(mu_sigma),
                             mu_sigma.numel() // 2, ptr(loss), ptr(dout), ptr(dml), ptr(ws), nb,
                             stream_ptr()), "sv_tvae_loss")
    return loss, dout, dml
