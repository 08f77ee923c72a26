"""INT8 refinement network -- TEST INFRASTRUCTURE ONLY.

The compression the paper plans (Sec. V: quantisation for speed and memory),
applied to the configurable network of ``vae.py`` at inference, written out
from its definition:

  * Weights, per output channel o: a_o = max |w[o]| (FP32), code =
    clamp(rint(w * (127 / a_o)), -127, 127), scale s_o = a_o / 127.
  * Activations, per tensor: every stored map records amax = max |stored
    value|; a layer whose input concatenates sources takes m = the largest of
    their amax values (x0: m_x0 = max(f * max d / 256, max I / 256)), and
    quantises each value it reads -- for a resized source the bilinear value
    computed in FP32 from the stored corners -- to clamp(rint(x * (127 / m)),
    -127, 127); zero padding is code 0.
  * Convolution: exact integer sum of code products, then
    y = float32(sum) * float32(s_in * s_o) + bias, leaky ReLU (slope 0.1),
    stored in BF16 (round to nearest even); the mu / logvar head stays FP32.
  * z = mu (inference only); the final layer is the FP32 network's, applied
    to the stored G0 (here in FP64).
Every scalar step above is an FP32 operation and is evaluated here in FP32 in
the same order, so the integer codes this produces are the method's codes.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import conv2d, resize
from .vae import make_input

F32 = np.float32
QMAX = 127


def bf16(x):
    """FP32 -> BF16 -> FP32, round to nearest even (no NaN inputs here)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def quantise(x, m):
    """Codes of values x (FP32) for a tensor whose amax is m (FP32)."""
    m = F32(m)
    inv = F32(QMAX) / m if m > 0 else F32(0)
    q = np.rint(np.asarray(x, np.float32) * inv)
    return np.clip(q, -QMAX, QMAX).astype(np.float32)


def input_scale(m):
    m = F32(m)
    return m / F32(QMAX)


def quantise_weights(w):
    """Per-output-channel codes and scales of FP32 OIHW weights."""
    w = np.asarray(w, np.float32)
    a = np.max(np.abs(w.reshape(w.shape[0], -1)), axis=1).astype(np.float32)
    inv = np.where(a > 0, F32(QMAX) / np.where(a > 0, a, F32(1)), F32(0)).astype(np.float32)
    q = np.clip(np.rint(w * inv[:, None, None, None]), -QMAX, QMAX).astype(np.float32)
    return q, (a / F32(QMAX)).astype(np.float32)


def f32_nearest(q):
    """The binary32 value nearest to the exact rational q (a Fraction), ties
    to the even significand: the rounding of IEEE 754 round-to-nearest.
    Found by exact comparison of q with the candidates around a first guess,
    so no intermediate rounding (e.g. through binary64) can shift it."""
    g = np.float32(float(q))
    cands = {g, np.nextafter(g, F32(np.inf)), np.nextafter(g, F32(-np.inf))}
    best = None
    for c in sorted(cands):
        dist = abs(Fraction(float(c)) - q)
        even = (int(np.asarray(c, np.float32).view(np.uint32)) & 1) == 0
        key = (dist, not even)
        if best is None or key < best[0]:
            best = (key, c)
    return F32(best[1])


def _bilin_axis(o, n_in, n_out):
    """Corner indices and FP32 weight along one axis of a resize from n_in to
    n_out samples with half-pixel centres: the exact source position is
    s = max(0, (o + 1/2) n_in / n_out - 1/2); i0 = floor(s), i1 = min(i0 + 1,
    n_in - 1), and the weight is the FP32 value nearest to s - i0."""
    s = (Fraction(2 * o + 1, 2) * n_in) / n_out - Fraction(1, 2)
    if s < 0:
        s = Fraction(0)
    i0 = math.floor(s)
    return i0, min(i0 + 1, n_in - 1), f32_nearest(s - i0)


def resize_f32(x, Ho, Wo):
    """Bilinear resize (half-pixel centres) evaluated in FP32 with the
    weights of _bilin_axis, in this order, every product and sum rounded to
    FP32 (no fused multiply-add): top = (1-lx) x00 + lx x01, bot = (1-lx) x10
    + lx x11 along the row, then (1-ly) top + ly bot down the column."""
    x = np.asarray(x, np.float32)
    Hi, Wi = x.shape[-2:]
    ys = [_bilin_axis(o, Hi, Ho) for o in range(Ho)]
    xs = [_bilin_axis(o, Wi, Wo) for o in range(Wo)]
    y0 = np.array([a for a, _, _ in ys]); y1 = np.array([b for _, b, _ in ys])
    ly = np.array([c for _, _, c in ys], np.float32)[:, None]
    x0 = np.array([a for a, _, _ in xs]); x1 = np.array([b for _, b, _ in xs])
    lx = np.array([c for _, _, c in xs], np.float32)[None, :]
    a00 = x[..., y0[:, None], x0[None, :]]
    a01 = x[..., y0[:, None], x1[None, :]]
    a10 = x[..., y1[:, None], x0[None, :]]
    a11 = x[..., y1[:, None], x1[None, :]]
    one = F32(1)
    top = (one - lx) * a00 + lx * a01
    bot = (one - lx) * a10 + lx * a11
    return ((one - ly) * top + ly * bot).astype(np.float32)


def qconv(x, m_in, w, b, stride, act, store_bf16=True):
    """One quantised layer on the values it reads (FP32 NCHW) with input amax
    m_in.  Returns (stored values, their amax, integer sums)."""
    xq = quantise(x, m_in)
    wq, sw = quantise_weights(w)
    k = wq.shape[-1]
    acc = conv2d(xq.astype(np.float64), wq.astype(np.float64), None, stride, (k - 1) // 2)
    acc = np.rint(acc).astype(np.int64)  # exact: integer products and sums below 2^53
    sc = (input_scale(m_in) * sw).astype(np.float32)
    val = acc.astype(np.float32) * sc[None, :, None, None] + np.asarray(b, np.float32)[None, :, None, None]
    if act:
        val = np.where(val > 0, val, F32(0.1) * val).astype(np.float32)
    out = bf16(val) if store_bf16 else val.astype(np.float32)
    return out, F32(np.max(np.abs(out))) if out.size else F32(0), acc


def forward(params, disp_low, img_low, factor, H, W):
    """INT8 inference of the configurable network; params as in vae.forward.
    Returns a dict with every stored map, its amax, mu / logvar and ``out``."""
    p = [(np.asarray(w, np.float32), np.asarray(b, np.float32)) for (w, b) in params]
    d = np.asarray(disp_low)
    im = np.asarray(img_low)
    if d.ndim == 2:
        d, im = d[None], im[None]
    x0 = np.stack([(F32(factor) / F32(256)) * d.astype(np.float32),
                   im.astype(np.float32) * F32(1.0 / 256)], axis=1).astype(np.float32)
    m_x0 = F32(x0.max()) if x0.size else F32(0)
    t = {"x0": x0, "amax_x0": m_x0}
    t["E1"], t["amax_E1"], _ = qconv(x0, m_x0, *p[0], 2, True)
    t["E2"], t["amax_E2"], _ = qconv(t["E1"], t["amax_E1"], *p[1], 2, True)
    t["E3"], t["amax_E3"], _ = qconv(t["E2"], t["amax_E2"], *p[2], 2, True)
    ml, t["amax_ML"], _ = qconv(t["E3"], t["amax_E3"], *p[3], 1, False, store_bf16=False)
    L = ml.shape[1] // 2
    t["mu"], t["logvar"] = ml[:, :L], ml[:, L:]
    t["G3"], t["amax_G3"], _ = qconv(t["mu"], t["amax_ML"], *p[4], 1, True)
    prev = "G3"
    for name, skip, li in (("G2", "E2", 5), ("G1", "E1", 6), ("G0", "x0", 7)):
        hs, ws = t[skip].shape[-2:]
        cat = np.concatenate([resize_f32(t[prev], hs, ws), t[skip]], axis=1)
        m = max(t["amax_" + prev], t["amax_" + skip])
        t[name], t["amax_" + name], _ = qconv(cat, m, *p[li], 1, True)
        prev = name
    # final layer: the FP32 network's, on the stored G0 (FP64 here)
    x064 = make_input(d, im, factor)
    catF = np.concatenate([t["G0"].astype(np.float64), x064], axis=1)
    wF, bF = params[8]
    up = resize(catF, H, W)
    R = conv2d(up, np.asarray(wF, np.float64), np.asarray(bF, np.float64), 1, 1)[:, 0]
    t["out"] = 256.0 * (resize(x064[:, 0], H, W) + R)
    return t
