"""FP64 StereoVAE network of Table I, as printed -- TEST INFRASTRUCTURE ONLY.

The refinement network exactly in the shape of Table I (Sec. III-B1):
feature extraction (FE), an encoder with two stride-2 downsamplings each
followed by a residual block R, a one-channel mu / sigma head with the
constant shifts of Eq. (8), a decoder with a 1x1 deconvolution, residual
blocks and two 5x5 stride-2 deconvolutions, skip connections, and one
upsampling layer to full resolution; plus the loss of Eqs. (9)-(11).
Composed from the FP64 primitives of ``oracle.c`` in the order the table
lists the layers.

Readings of the paper taken here (each is also listed in the design notes):
  * X_0 is the coarse disparity and X_1 the reduced left image, both divided
    by 256 (the disparity in full-resolution pixels: factor * d / 256).
  * Every layer is a 5x5 convolution with padding 2 (stride 2 where the
    table halves the size) except the 1x1 head and the 1x1 deconvolution.
  * A residual block R is one 5x5 stride-1 convolution whose output is
    concatenated with its input, as the table's "A & A_R" inputs show.
  * "&" is channel concatenation in the order the table writes it.
  * Leaky ReLU (slope 0.1) after every layer except the mu / sigma head and
    the final upsampling layer, which are linear.
  * Deconvolution = transposed convolution with kernel k, stride s and
    padding (k - 1) / 2, its output cut to the size of the level it feeds
    (the skip map's size, or H x W for the last layer: the output-padding
    choice that makes odd sizes come out exactly).  The final upsampling layer
    has stride equal to the reduction factor f (2 in Table I).
  * Eq. (8): z = (mu - 1) + eps * exp(sigma - 1), so exp(sigma - 1) is a
    standard deviation; at inference eps = 0, z = mu - 1.
  * Eq. (11) read as the KL divergence of N(mu - 1, exp(sigma - 1)^2) from
    N(0, 1): 0.5 * ((mu - 1)^2 - 1 + exp(2 (sigma - 1)) - 2 (sigma - 1)),
    averaged over latent positions.
  * Eq. (10): absolute errors against the non-occluded and the all-pixel
    ground truth, each summed over its mask and both divided by the number of
    all-pixel ground-truth points, so non-occluded points weigh twice;
    Eq. (9): total = 256 * (Loss_1 + Loss_2) with Y and the ground truth in
    units of 256 px.
"""
from __future__ import annotations

import numpy as np

from . import conv2d, conv2d_dw, conv2d_dx, tconv2d

SLOPE = 0.1
K = 5
# (name, out channels, in channels, kernel, stride (0: the factor f), transposed)
LAYERS = (
    ("FE_1", 32, 1, 5, 1, False),
    ("FE_2", 32, 1, 5, 1, False),
    ("EN_1", 16, 64, 5, 2, False),
    ("EN_1_R", 8, 16, 5, 1, False),
    ("EN_2", 32, 24, 5, 2, False),
    ("EN_2_R", 16, 32, 5, 1, False),
    ("MS", 2, 48, 1, 1, False),
    ("D_1", 32, 1, 1, 1, True),
    ("D_1_R", 16, 80, 5, 1, False),
    ("D_2", 16, 96, 5, 2, True),
    ("D_2_R", 8, 40, 5, 1, False),
    ("D", 16, 48, 5, 2, True),
    ("Y", 1, 81, 5, 0, True),
)
NAMES = tuple(l[0] for l in LAYERS)


def layer_shapes():
    """(out, in, k) per layer in canonical order."""
    return [(o, i, k) for (_, o, i, k, _, _) in LAYERS]


def n_params() -> int:
    return sum(o * i * k * k + o for (o, i, k) in layer_shapes())


def lrelu(x):
    return np.where(x > 0, x, SLOPE * x)


def flatten(params):
    return np.concatenate([np.concatenate([np.ravel(w), np.ravel(b)]) for (w, b) in params])


def unflatten(vec):
    out, o = [], 0
    for (co, ci, k) in layer_shapes():
        n = co * ci * k * k
        out.append((np.asarray(vec[o:o + n], np.float64).reshape(co, ci, k, k),
                    np.asarray(vec[o + n:o + n + co], np.float64)))
        o += n + co
    return out


def _conv(x, wb, stride):
    w, b = wb
    k = w.shape[-1]
    return conv2d(x, w, b, stride, (k - 1) // 2)


def _deconv(x, wb, stride, Ho, Wo):
    w, b = wb
    k = w.shape[-1]
    return tconv2d(x, w, b, stride, (k - 1) // 2, Ho, Wo)


def cat(*xs):
    return np.concatenate(xs, axis=1)


def forward(params, disp_low, img_low, factor, H, W, eps=None):
    """Table I forward.  params: list of (w [O][C][k][k], b) in LAYERS order.
    disp_low, img_low: uint8 [B][h][w] (coarse disparity in reduced px and the
    reduced left image); eps: [B][1][h/4][w/4] or None.  Returns a dict of every
    map; ``out`` is the disparity in full-resolution px, [B][H][W]."""
    p = dict(zip(NAMES, [(np.asarray(w, np.float64), np.asarray(b, np.float64)) for (w, b) in params]))
    d = np.asarray(disp_low, np.float64)
    im = np.asarray(img_low, np.float64)
    if d.ndim == 2:
        d, im = d[None], im[None]
    t = {"X_0": (factor * d / 256.0)[:, None], "X_1": (im / 256.0)[:, None]}
    # feature extraction
    t["FE_1"] = lrelu(_conv(t["X_0"], p["FE_1"], 1))
    t["FE_2"] = lrelu(_conv(t["X_1"], p["FE_2"], 1))
    # encoder
    t["EN_1"] = lrelu(_conv(cat(t["FE_1"], t["FE_2"]), p["EN_1"], 2))
    t["EN_1_R"] = lrelu(_conv(t["EN_1"], p["EN_1_R"], 1))
    t["EN_2"] = lrelu(_conv(cat(t["EN_1"], t["EN_1_R"]), p["EN_2"], 2))
    t["EN_2_R"] = lrelu(_conv(t["EN_2"], p["EN_2_R"], 1))
    ms = _conv(cat(t["EN_2"], t["EN_2_R"]), p["MS"], 1)
    t["mu"], t["sigma"] = ms[:, 0:1], ms[:, 1:2]
    # Eq. (8)
    t["z"] = t["mu"] - 1.0
    if eps is not None:
        t["eps"] = np.asarray(eps, np.float64).reshape(t["mu"].shape)
        t["z"] = t["z"] + t["eps"] * np.exp(t["sigma"] - 1.0)
    # decoder
    h2, w2 = t["EN_1"].shape[-2:]
    h1, w1 = t["FE_1"].shape[-2:]
    t["D_1"] = lrelu(_deconv(t["z"], p["D_1"], 1, *t["z"].shape[-2:]))
    t["D_1_R"] = lrelu(_conv(cat(t["D_1"], t["EN_2"], t["EN_2_R"]), p["D_1_R"], 1))
    t["D_2"] = lrelu(_deconv(cat(t["D_1"], t["EN_2"], t["EN_2_R"], t["D_1_R"]), p["D_2"], 2, h2, w2))
    t["D_2_R"] = lrelu(_conv(cat(t["D_2"], t["EN_1"], t["EN_1_R"]), p["D_2_R"], 1))
    t["D"] = lrelu(_deconv(cat(t["D_2"], t["EN_1"], t["EN_1_R"], t["D_2_R"]), p["D"], 2, h1, w1))
    # upsampling to full resolution
    t["Y"] = _deconv(cat(t["D"], t["X_0"], t["FE_1"], t["FE_2"]), p["Y"], factor, H, W)[:, 0]
    t["out"] = 256.0 * t["Y"]
    t["factor"] = factor
    return t


def loss(out, gt, noc, occ, mu, sigma):
    """Eqs. (9)-(11) in the reading above.  out, gt: [B][H][W] in px; noc, occ:
    bool masks of the two ground truths; mu, sigma: the head's maps.  Returns
    (total, 256 * Loss_1, 256 * Loss_2, dtotal/dout, dtotal/dmu, dtotal/dsigma);
    the derivative of |e| at e = 0 is taken as 0."""
    out = np.asarray(out, np.float64)
    gt = np.asarray(gt, np.float64)
    noc = np.asarray(noc, bool)
    occ = np.asarray(occ, bool)
    n = max(int(occ.sum()), 1)
    # 256 * |gt/256 - Y| = |gt - out| in px
    e = out - gt
    l1 = (np.abs(e)[noc].sum() + np.abs(e)[occ].sum()) / n
    dout = (np.sign(e) * noc + np.sign(e) * occ) / n
    m = np.asarray(mu, np.float64) - 1.0
    s = np.asarray(sigma, np.float64) - 1.0
    nl = m.size
    l2 = 256.0 * np.sum(0.5 * (m * m - 1.0 + np.exp(2.0 * s) - 2.0 * s)) / nl
    dmu = 256.0 * m / nl
    dsigma = 256.0 * (np.exp(2.0 * s) - 1.0) / nl
    return l1 + l2, l1, l2, dout, dmu, dsigma


# ---- adjoint ---------------------------------------------------------------------
# (name, inputs in "&" order, stride (0: the factor), transposed, activation)
_GRAPH = (
    ("FE_1", ("X_0",), 1, False, True),
    ("FE_2", ("X_1",), 1, False, True),
    ("EN_1", ("FE_1", "FE_2"), 2, False, True),
    ("EN_1_R", ("EN_1",), 1, False, True),
    ("EN_2", ("EN_1", "EN_1_R"), 2, False, True),
    ("EN_2_R", ("EN_2",), 1, False, True),
    ("MS", ("EN_2", "EN_2_R"), 1, False, False),
    ("D_1", ("z",), 1, True, True),
    ("D_1_R", ("D_1", "EN_2", "EN_2_R"), 1, False, True),
    ("D_2", ("D_1", "EN_2", "EN_2_R", "D_1_R"), 2, True, True),
    ("D_2_R", ("D_2", "EN_1", "EN_1_R"), 1, False, True),
    ("D", ("D_2", "EN_1", "EN_1_R", "D_2_R"), 2, True, True),
    ("Y", ("D", "X_0", "FE_1", "FE_2"), 0, True, False),
)


def backward(params, t, dout, dmu=None, dsigma=None):
    """Adjoint of ``forward`` for the scalar sum(dout * out) + sum(dmu * mu) +
    sum(dsigma * sigma) (the loss's gradients plug in as dout, dmu, dsigma).
    Returns (dw, db) per layer in LAYERS order.  The leaky ReLU's derivative
    is taken from the sign of the stored output (0.1 at exactly 0)."""
    p = dict(zip(NAMES, [(np.asarray(w, np.float64), np.asarray(b, np.float64)) for (w, b) in params]))
    g = {}

    def acc(name, v):
        g[name] = g.get(name, 0.0) + v

    acc("Y", 256.0 * np.asarray(dout, np.float64)[:, None])
    grads = {}
    factor = t["factor"]
    for (name, ins, stride, transposed, act) in reversed(_GRAPH):
        w, b = p[name]
        k = w.shape[-1]
        pad = (k - 1) // 2
        s = factor if stride == 0 else stride
        if name == "MS":
            dm = g.get("mu_z", 0.0) + (0.0 if dmu is None else np.asarray(dmu, np.float64).reshape(t["mu"].shape))
            ds = g.get("sigma_z", 0.0) + (0.0 if dsigma is None else np.asarray(dsigma, np.float64).reshape(t["sigma"].shape))
            dy = np.concatenate([np.broadcast_to(dm, t["mu"].shape), np.broadcast_to(ds, t["sigma"].shape)], axis=1)
        else:
            dy = g.get(name)
            if dy is None:
                dy = np.zeros_like(t[name] if name != "Y" else t["Y"][:, None])
            if act:
                dy = dy * np.where(t[name] > 0, 1.0, SLOPE)
        x = cat(*[t[i] for i in ins])
        if transposed:
            # y = tconv(x): dW from the strided correlation of dy against x, dx = conv(dy; W^T)
            dwt, _ = conv2d_dw(dy, x, k, s, pad)          # [C][O][k][k]
            dw = np.ascontiguousarray(dwt.transpose(1, 0, 2, 3))
            dx = conv2d(dy, np.ascontiguousarray(w.transpose(1, 0, 2, 3)), None, s, pad)
        else:
            dw, _ = conv2d_dw(x, dy, k, s, pad)
            dx = conv2d_dx(dy, w, x.shape, s, pad)
        grads[name] = (dw, dy.sum(axis=(0, 2, 3)))
        c0 = 0
        for i in ins:
            c = t[i].shape[1]
            if i == "z":
                dz = dx[:, c0:c0 + c]
                g["mu_z"] = dz
                g["sigma_z"] = dz * t["eps"] * np.exp(t["sigma"] - 1.0) if "eps" in t else np.zeros_like(dz)
            elif i not in ("X_0", "X_1"):
                acc(i, dx[:, c0:c0 + c])
            c0 += c
    return [grads[n] for n in NAMES]
