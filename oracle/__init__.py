"""CPU oracle for the StereoVAE hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of what the GPU library
computes: integer downsample / census / Hamming cost / winner-take-all
(``oracle.c``), and an FP64 refinement network composed from FP64 primitives
(``vae.py``).  Only ``tests/``, the smoke check and the benchmark's CPU
baseline may import it; the product path never does.  It imports nothing from
the GPU package and the GPU package imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared",
                               "-fPIC", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        _lib = ctypes.CDLL(_SO)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def downsample(img: np.ndarray, f: int) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    if img.ndim == 2:
        img = img[None]
    B, H, W = img.shape
    h, w = -(-H // f), -(-W // f)
    out = np.empty((B, h, w), dtype=np.uint8)
    lib().or_downsample(_p(img), B, H, W, W, f, _p(out))
    return out


def census(low: np.ndarray, win_w: int, win_h: int) -> np.ndarray:
    low = np.ascontiguousarray(low, dtype=np.uint8)
    if low.ndim == 2:
        low = low[None]
    B, h, w = low.shape
    out = np.empty((B, h, w), dtype=np.uint64)
    lib().or_census(_p(low), B, h, w, win_w, win_h, _p(out))
    return out


def cost_volume(cl: np.ndarray, cr: np.ndarray, D: int, nbits: int) -> np.ndarray:
    cl = np.ascontiguousarray(cl, dtype=np.uint64)
    cr = np.ascontiguousarray(cr, dtype=np.uint64)
    B, h, w = cl.shape
    out = np.empty((B, h, w, D), dtype=np.int32)
    lib().or_cost_volume(_p(cl), _p(cr), B, h, w, D, nbits, _p(out))
    return out


def wta(cost: np.ndarray) -> np.ndarray:
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    B, h, w, D = cost.shape
    out = np.empty((B, h, w), dtype=np.uint8)
    lib().or_wta(_p(cost), B, h, w, D, _p(out))
    return out


def match(left: np.ndarray, right: np.ndarray, f: int, win_w: int, win_h: int, D: int):
    """Coarse matching stage: (low-res left image, census L, census R, disparity)."""
    lo_l, lo_r = downsample(left, f), downsample(right, f)
    cl, cr = census(lo_l, win_w, win_h), census(lo_r, win_w, win_h)
    nbits = win_w * win_h - 1
    disp = wta(cost_volume(cl, cr, D, nbits))
    return lo_l, cl, cr, disp


def sgm_path(cost: np.ndarray, P1: int, P2: int, direction: int) -> np.ndarray:
    """Path cost of Eq. (4) along one direction (0 L->R, 1 R->L, 2 T->B, 3 B->T)."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    B, h, w, D = cost.shape
    out = np.empty_like(cost)
    lib().or_sgm_path(_p(cost), B, h, w, D, P1, P2, direction, _p(out))
    return out


def sgm(cost: np.ndarray, P1: int, P2: int) -> np.ndarray:
    """Aggregated cost of Eq. (5) over the four axis directions."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    B, h, w, D = cost.shape
    out = np.empty_like(cost)
    scratch = np.empty_like(cost)
    lib().or_sgm(_p(cost), B, h, w, D, P1, P2, _p(out), _p(scratch))
    return out


def smp(disp: np.ndarray, D: int) -> np.ndarray:
    """Single matching phase of Eq. (7) with nearest-valid filling."""
    disp = np.ascontiguousarray(disp, dtype=np.uint8)
    if disp.ndim == 2:
        disp = disp[None]
    B, h, w = disp.shape
    assert w <= 1 << 16
    out = np.empty_like(disp)
    lib().or_smp(_p(disp), B, h, w, D, _p(out))
    return out


def median3(disp: np.ndarray) -> np.ndarray:
    """3 x 3 median filter, borders replicated."""
    disp = np.ascontiguousarray(disp, dtype=np.uint8)
    if disp.ndim == 2:
        disp = disp[None]
    B, h, w = disp.shape
    out = np.empty_like(disp)
    lib().or_median3(_p(disp), B, h, w, _p(out))
    return out


def zncc_cost(low_l: np.ndarray, low_r: np.ndarray, D: int, win_w: int, win_h: int) -> np.ndarray:
    """Quantised ZNCC cost of Eqs. (1)-(3): floor(32 C + 1/2), int32 [B, h, w, D]."""
    low_l = np.ascontiguousarray(low_l, dtype=np.uint8)
    low_r = np.ascontiguousarray(low_r, dtype=np.uint8)
    if low_l.ndim == 2:
        low_l, low_r = low_l[None], low_r[None]
    B, h, w = low_l.shape
    out = np.empty((B, h, w, D), dtype=np.int32)
    lib().or_zncc_cost(_p(low_l), _p(low_r), B, h, w, D, win_w, win_h, _p(out))
    return out


def match_zncc_sgm(left: np.ndarray, right: np.ndarray, f: int, win_w: int, win_h: int, D: int,
                   P1: int, P2: int):
    """ZNCC + SGM + WTA + SMP + median (the paper's main coarse pipeline):
    (low-res left image, raw disparity, post-processed disparity)."""
    lo_l, lo_r = downsample(left, f), downsample(right, f)
    raw = wta(sgm(zncc_cost(lo_l, lo_r, D, win_w, win_h), P1, P2))
    return lo_l, raw, median3(smp(raw, D))


def match_sgm(left: np.ndarray, right: np.ndarray, f: int, win_w: int, win_h: int, D: int,
              P1: int, P2: int):
    """Census + SGM + WTA + SMP + median: (low-res left image, raw SGM disparity,
    post-processed disparity)."""
    lo_l, lo_r = downsample(left, f), downsample(right, f)
    cl, cr = census(lo_l, win_w, win_h), census(lo_r, win_w, win_h)
    nbits = win_w * win_h - 1
    raw = wta(sgm(cost_volume(cl, cr, D, nbits), P1, P2))
    return lo_l, raw, median3(smp(raw, D))


def conv2d(x, wt, bias, stride, pad):
    x = np.ascontiguousarray(x, dtype=np.float64)
    wt = np.ascontiguousarray(wt, dtype=np.float64)
    B, C, H, W = x.shape
    O, C2, k, k2 = wt.shape
    assert C2 == C and k == k2
    Ho, Wo = (H + 2 * pad - k) // stride + 1, (W + 2 * pad - k) // stride + 1
    y = np.empty((B, O, Ho, Wo), dtype=np.float64)
    bp = None
    if bias is not None:
        bias = np.ascontiguousarray(bias, dtype=np.float64)
        bp = _p(bias)
    lib().or_conv2d(_p(x), B, C, H, W, _p(wt), bp, O, k, stride, pad, _p(y))
    return y


def conv2d_dx(dy, wt, x_shape, stride, pad):
    dy = np.ascontiguousarray(dy, dtype=np.float64)
    wt = np.ascontiguousarray(wt, dtype=np.float64)
    B, C, H, W = x_shape
    O, _, k, _ = wt.shape
    dx = np.empty((B, C, H, W), dtype=np.float64)
    lib().or_conv2d_dx(_p(dy), B, C, H, W, _p(wt), O, k, stride, pad, _p(dx))
    return dx


def conv2d_dw(x, dy, k, stride, pad):
    x = np.ascontiguousarray(x, dtype=np.float64)
    dy = np.ascontiguousarray(dy, dtype=np.float64)
    B, C, H, W = x.shape
    O = dy.shape[1]
    dw = np.empty((O, C, k, k), dtype=np.float64)
    db = np.empty(O, dtype=np.float64)
    lib().or_conv2d_dw(_p(x), _p(dy), B, C, H, W, O, k, stride, pad, _p(dw), _p(db))
    return dw, db


def tconv2d(x, wt, bias, stride, pad, Ho, Wo):
    """Transposed convolution, weights [O][C][k][k]; output Ho x Wo (see or_tconv2d)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    wt = np.ascontiguousarray(wt, dtype=np.float64)
    B, C, H, W = x.shape
    O, C2, k, k2 = wt.shape
    assert C2 == C and k == k2
    y = np.empty((B, O, Ho, Wo), dtype=np.float64)
    bp = None
    if bias is not None:
        bias = np.ascontiguousarray(bias, dtype=np.float64)
        bp = _p(bias)
    lib().or_tconv2d(_p(x), B, C, H, W, _p(wt), bp, O, k, stride, pad, Ho, Wo, _p(y))
    return y


def resize(x, Ho, Wo):
    x = np.ascontiguousarray(x, dtype=np.float64)
    lead = x.shape[:-2]
    Hi, Wi = x.shape[-2:]
    N = int(np.prod(lead)) if lead else 1
    y = np.empty(lead + (Ho, Wo), dtype=np.float64)
    lib().or_resize_bilinear(_p(x), N, Hi, Wi, Ho, Wo, _p(y))
    return y


def resize_adj(dy, Hi, Wi):
    dy = np.ascontiguousarray(dy, dtype=np.float64)
    lead = dy.shape[:-2]
    Ho, Wo = dy.shape[-2:]
    N = int(np.prod(lead)) if lead else 1
    dx = np.empty(lead + (Hi, Wi), dtype=np.float64)
    lib().or_resize_bilinear_adj(_p(dy), N, Hi, Wi, Ho, Wo, _p(dx))
    return dx
