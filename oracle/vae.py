"""FP64 refinement network of the oracle -- TEST INFRASTRUCTURE ONLY.

Composes the FP64 primitives of ``oracle.c`` into the tiny VAE that upsamples
and refines the coarse disparity map (Sec. III-B, Table I), its loss
(Sec. III-B2, Eqs. (9)-(11), in the reading below) and its exact adjoint, plus
one Adam step (Sec. IV-A).  Layer by layer, in the order the network runs.

Readings of the paper taken here (each is also listed in the design notes):
  * Architecture: encoder of three 3x3 stride-2 convolutions (2 -> C1 -> C2 -> C3),
    a 1x1 head giving mu and log-variance (L channels each), a 1x1 decoder
    input layer, three decoder levels that each bilinearly resize to the next
    encoder level, concatenate that level's encoder map (skip connection) and
    apply a 3x3 convolution, then a final layer that resizes [G0, x0] to full
    resolution and applies a 3x3 convolution to one channel.  Table I's
    5x5 kernels, FE module and residual blocks are replaced by this shape.
  * Leaky ReLU slope 0.1 (Sec. III-B1); its derivative at exactly 0 is taken as 0.1.
  * Reparameterisation in the standard form z = mu + eps * exp(logvar / 2)
    (Eq. (8) without the constant shifts, which a bias of the head absorbs);
    at inference z = mu.
  * KL divergence to N(0, I) in the standard form, averaged over latent
    elements (Eq. (11) is garbled in the source).
  * Inputs normalised by 1/256 and the output scaled back by 256 (Sec. III-B2).
  * Output is a residual over the linear upscaling of the coarse map
    ("Mini+Linear", Sec. IV-C): Y = resize(x0[:, 0]) + R.
  * Data term: smooth-L1 (beta = 1 px) mean over pixels; loss = data + w_kl * KL.
"""
from __future__ import annotations

import numpy as np

from . import conv2d, conv2d_dx, conv2d_dw, resize, resize_adj

SLOPE = 0.1
LAYERS = ("E1", "E2", "E3", "HEAD", "G3", "G2", "G1", "G0", "F")


def layer_shapes(c1: int, c2: int, c3: int, latent: int):
    """(out_ch, in_ch, k, stride) per layer, in execution order."""
    return [
        (c1, 2, 3, 2),             # E1
        (c2, c1, 3, 2),            # E2
        (c3, c2, 3, 2),            # E3
        (2 * latent, c3, 1, 1),    # HEAD -> [mu | logvar]
        (c3, latent, 1, 1),        # G3
        (c2, c3 + c2, 3, 1),       # G2 on [resize(G3), E2]
        (c1, c2 + c1, 3, 1),       # G1 on [resize(G2), E1]
        (c1, c1 + 2, 3, 1),        # G0 on [resize(G1), x0]
        (1, c1 + 2, 3, 1),         # F  on resize([G0, x0]) at full resolution
    ]


def n_params(c1, c2, c3, latent) -> int:
    return sum(o * i * k * k + o for (o, i, k, s) in layer_shapes(c1, c2, c3, latent))


def lrelu(x):
    return np.where(x > 0, x, SLOPE * x)


def lrelu_grad(pre):
    return np.where(pre > 0, 1.0, SLOPE)


def _conv(x, wb, stride):
    w, b = wb
    k = w.shape[-1]
    return conv2d(x, w, b, stride, (k - 1) // 2)


def make_input(disp_low, img_low, factor):
    """x0 = [factor * d / 256, I / 256], NCHW float64."""
    d = np.asarray(disp_low, dtype=np.float64)
    im = np.asarray(img_low, dtype=np.float64)
    if d.ndim == 2:
        d, im = d[None], im[None]
    return np.stack([factor * d / 256.0, im / 256.0], axis=1)


def forward(params, disp_low, img_low, factor, H, W, eps=None):
    """Network forward.  params: list of (w OIHW, b) per layer.  Returns a dict
    of every intermediate; ``out`` is the refined disparity in full-res px."""
    p = [(np.asarray(w, np.float64), np.asarray(b, np.float64)) for (w, b) in params]
    x0 = make_input(disp_low, img_low, factor)
    t = {"x0": x0}
    t["E1pre"] = _conv(x0, p[0], 2)
    t["E1"] = lrelu(t["E1pre"])
    t["E2pre"] = _conv(t["E1"], p[1], 2)
    t["E2"] = lrelu(t["E2pre"])
    t["E3pre"] = _conv(t["E2"], p[2], 2)
    t["E3"] = lrelu(t["E3pre"])
    ml = _conv(t["E3"], p[3], 1)
    L = ml.shape[1] // 2
    t["mu"], t["logvar"] = ml[:, :L], ml[:, L:]
    if eps is None:
        t["z"] = t["mu"]
    else:
        t["eps"] = np.asarray(eps, np.float64)
        t["z"] = t["mu"] + t["eps"] * np.exp(0.5 * t["logvar"])
    t["G3pre"] = _conv(t["z"], p[4], 1)
    t["G3"] = lrelu(t["G3pre"])
    prev = t["G3"]
    for name, skip, li in (("G2", "E2", 5), ("G1", "E1", 6), ("G0", "x0", 7)):
        hs, ws = t[skip].shape[-2:]
        cat = np.concatenate([resize(prev, hs, ws), t[skip]], axis=1)
        t[name + "cat"] = cat
        t[name + "pre"] = _conv(cat, p[li], 1)
        t[name] = lrelu(t[name + "pre"])
        prev = t[name]
    catF = np.concatenate([t["G0"], x0], axis=1)
    t["Fcat_up"] = resize(catF, H, W)
    t["R"] = _conv(t["Fcat_up"], p[8], 1)[:, 0]
    t["base"] = resize(x0[:, 0], H, W)
    t["Y"] = t["base"] + t["R"]
    t["out"] = 256.0 * t["Y"]
    return t


def kl_divergence(mu, logvar):
    """Mean over latent elements of KL(N(mu, exp(logvar)) || N(0, 1))."""
    return float(np.mean(0.5 * (mu ** 2 + np.exp(logvar) - 1.0 - logvar)))


def smooth_l1(out, gt):
    """Mean smooth-L1 (beta = 1 px) and its gradient with respect to out."""
    e = np.asarray(out, np.float64) - np.asarray(gt, np.float64)
    a = np.abs(e)
    loss = np.where(a < 1.0, 0.5 * e * e, a - 0.5)
    return float(np.mean(loss)), np.clip(e, -1.0, 1.0) / e.size


def loss(t, gt, kl_weight):
    data, dout = smooth_l1(t["out"], gt)
    kl = kl_divergence(t["mu"], t["logvar"])
    return data + kl_weight * kl, data, kl, dout


def backward(params, t, dout, kl_weight):
    """Adjoint of ``forward`` for the loss  sum(dout * out) + kl_weight * KL.

    Returns the list of (dw, db) per layer, in layer order."""
    p = [(np.asarray(w, np.float64), np.asarray(b, np.float64)) for (w, b) in params]
    g = [None] * 9
    x0 = t["x0"]
    C1 = t["G0"].shape[1]
    dY = 256.0 * np.asarray(dout, np.float64)
    dR = dY[:, None]
    # final layer: R = conv3x3(resize([G0, x0]))
    g[8] = conv2d_dw(t["Fcat_up"], dR, 3, 1, 1)
    dcat_up = conv2d_dx(dR, p[8][0], t["Fcat_up"].shape, 1, 1)
    dcat = resize_adj(dcat_up, *x0.shape[-2:])
    dprev = dcat[:, :C1]
    dskip = {}
    # decoder levels, last to first
    for name, skip, li in (("G0", "x0", 7), ("G1", "E1", 6), ("G2", "E2", 5)):
        dpre = dprev * lrelu_grad(t[name + "pre"])
        g[li] = conv2d_dw(t[name + "cat"], dpre, 3, 1, 1)
        dcat = conv2d_dx(dpre, p[li][0], t[name + "cat"].shape, 1, 1)
        nprev = dcat.shape[1] - t[skip].shape[1]
        dskip[skip] = dcat[:, nprev:]
        below = {"G0": "G1", "G1": "G2", "G2": "G3"}[name]
        dprev = resize_adj(dcat[:, :nprev], *t[below].shape[-2:])
    # G3 = lrelu(conv1x1(z))
    dpre = dprev * lrelu_grad(t["G3pre"])
    g[4] = conv2d_dw(t["z"], dpre, 1, 1, 0)
    dz = conv2d_dx(dpre, p[4][0], t["z"].shape, 1, 0)
    # latent: reparameterisation and KL
    mu, lv = t["mu"], t["logvar"]
    n_lat = mu.size
    dmu = dz + kl_weight * mu / n_lat
    dlv = kl_weight * 0.5 * (np.exp(lv) - 1.0) / n_lat
    if "eps" in t:
        dlv = dlv + dz * t["eps"] * 0.5 * np.exp(0.5 * lv)
    dml = np.concatenate([dmu, dlv], axis=1)
    g[3] = conv2d_dw(t["E3"], dml, 1, 1, 0)
    dE3 = conv2d_dx(dml, p[3][0], t["E3"].shape, 1, 0)
    # encoder, last to first; the skip gradients join here
    dpre = dE3 * lrelu_grad(t["E3pre"])
    g[2] = conv2d_dw(t["E2"], dpre, 3, 2, 1)
    dE2 = conv2d_dx(dpre, p[2][0], t["E2"].shape, 2, 1) + dskip["E2"]
    dpre = dE2 * lrelu_grad(t["E2pre"])
    g[1] = conv2d_dw(t["E1"], dpre, 3, 2, 1)
    dE1 = conv2d_dx(dpre, p[1][0], t["E1"].shape, 2, 1) + dskip["E1"]
    dpre = dE1 * lrelu_grad(t["E1pre"])
    g[0] = conv2d_dw(x0, dpre, 3, 2, 1)
    return g


def adam_step(w, grad, m, v, step, lr=5e-4, beta1=0.99, beta2=0.999, eps=1e-8):
    """One Adam update (Sec. IV-A hyper-parameters; eps is not given in the paper).

    Returns the new (w, m, v); step counts from 1."""
    w, grad, m, v = (np.asarray(a, np.float64) for a in (w, grad, m, v))
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def flatten(params):
    """Canonical parameter vector: per layer, weights (OIHW) then bias."""
    return np.concatenate([np.concatenate([np.ravel(w), np.ravel(b)]) for (w, b) in params])


def unflatten(vec, c1, c2, c3, latent):
    out, o = [], 0
    for (co, ci, k, s) in layer_shapes(c1, c2, c3, latent):
        n = co * ci * k * k
        w = np.asarray(vec[o:o + n]).reshape(co, ci, k, k)
        o += n
        b = np.asarray(vec[o:o + co])
        o += co
        out.append((w, b))
    assert o == len(vec)
    return out
