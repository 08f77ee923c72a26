"""Seeded stereo-pair, weight and noise generators.

Every draw comes from ``numpy.random.Generator(PCG64(seed))`` so a seed fixes
the input bit for bit.  The recipe (blurred-noise texture, planar Voronoi
disparity cells, z-buffered forward warp, hole fill, sensor noise) stands in
for the KITTI 2015 driving scenes the paper evaluates on (Sec. IV-A): it keeps
their image size and disparity range but reproduces no item of that dataset.
"""
from __future__ import annotations

import dataclasses

import numpy as np

# The five workload presets.  Shapes, factors and windows per preset; sizes of
# the uneven batch are drawn in gen_preset.
# Workload presets; pair `index` of a preset has seed seed0 + index.
PRESETS = {
    "pair256x128": dict(seed0=1000, H=128, W=256, n_cells=6, dmin=4.0, dmax=24.0, factor=2, win_w=5,
                        win_h=5, D=16, channels=(16, 32, 64), latent=64, batch=1),
    "pair1242x375": dict(seed0=2000, H=375, W=1242, n_cells=18, dmin=0.0, dmax=190.0, factor=4, win_w=9,
                         win_h=7, D=48, channels=(32, 64, 128), latent=128, batch=1),
    "batch8_256x128": dict(seed0=3000, H=128, W=256, n_cells=6, dmin=4.0, dmax=24.0, factor=2, win_w=5,
                           win_h=5, D=16, channels=(16, 32, 64), latent=64, batch=8),
    "uneven64": dict(seed0=4000, n_cells=18, factor=4, win_w=9, win_h=7, channels=(32, 64, 128), latent=128,
                     batch=64),
    "crops512x256": dict(seed0=5000, H=256, W=512, n_cells=6, dmin=4.0, dmax=24.0, factor=2, win_w=5,
                         win_h=5, D=16, channels=(16, 32, 64), latent=64, batch=16),
}


@dataclasses.dataclass
class StereoPair:
    left: np.ndarray    # uint8 [H, W]
    right: np.ndarray   # uint8 [H, W]
    gt: np.ndarray      # float32 [H, W], disparity in full-res px (left is the reference)
    noc: np.ndarray     # bool [H, W], left pixel visible in the right view
    occ: np.ndarray     # bool [H, W], pixel has ground truth (dense: all True)
    D: int = 0          # low-res disparity range the pair is matched over (0: preset's)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _gauss_taps(sigma: float, radius: int) -> np.ndarray:
    x = np.arange(-radius, radius + 1, dtype=np.float64)
    k = np.exp(-0.5 * (x / sigma) ** 2)
    return k / k.sum()


def _blur(img: np.ndarray, sigma: float = 1.5, radius: int = 5) -> np.ndarray:
    """Separable Gaussian blur with mirror ('reflect') borders."""
    k = _gauss_taps(sigma, radius)
    H, W = img.shape
    p = np.pad(img, ((radius, radius), (0, 0)), mode="reflect")
    t = np.zeros((H, W))
    for i in range(2 * radius + 1):
        t += k[i] * p[i:i + H, :]
    p = np.pad(t, ((0, 0), (radius, radius)), mode="reflect")
    out = np.zeros((H, W))
    for i in range(2 * radius + 1):
        out += k[i] * p[:, i:i + W]
    return out


def _texture(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    return _blur(rng.uniform(0.0, 255.0, size=(H, W)))


def _quantise(x: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def _planar_cells(rng, H, W, n_cells, dmin, dmax):
    """Voronoi cells, each carrying an exact plane that stays inside [dmin, dmax]."""
    seeds = rng.uniform(0.0, 1.0, size=(n_cells, 2)) * np.array([W, H], dtype=np.float64)
    d0 = rng.uniform(dmin, dmax, size=n_cells)
    slopes = rng.uniform(-0.05, 0.05, size=(n_cells, 2))
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    # nearest seed wins; argmin keeps the lowest index on exact ties
    dist = np.stack([(xs - sx) ** 2 + (ys - sy) ** 2 for sx, sy in seeds])
    label = np.argmin(dist, axis=0)
    disp = np.zeros((H, W))
    for c in range(n_cells):
        m = label == c
        if not m.any():
            continue
        sx, sy = seeds[c]
        g = slopes[c, 0] * (xs[m] - sx) + slopes[c, 1] * (ys[m] - sy)
        t = 1.0
        pos, neg = g > 0, g < 0
        if pos.any():
            t = min(t, float(np.min((dmax - d0[c]) / g[pos])))
        if neg.any():
            t = min(t, float(np.min((dmin - d0[c]) / g[neg])))
        t = max(0.0, t) * (1.0 - 1e-9)
        disp[m] = d0[c] + t * g
    assert disp.min() >= dmin - 1e-6 and disp.max() <= dmax + 1e-6
    return np.clip(disp, dmin, dmax)


def _forward_warp(left: np.ndarray, disp: np.ndarray):
    """Move each left pixel to x' = floor(x - d + 1/2); larger d wins, then the first writer."""
    H, W = left.shape
    ys, xs = np.mgrid[0:H, 0:W]
    xt = np.floor(xs - disp + 0.5).astype(np.int64)
    valid = (xt >= 0) & (xt < W)
    idx = (ys * W + xs).ravel()
    tgt = (ys * W + xt).ravel()
    d = disp.ravel()
    v = valid.ravel()
    idx, tgt, d = idx[v], tgt[v], d[v]
    order = np.lexsort((idx, -d, tgt))       # by target, then larger d, then row-major order
    tgt_sorted = tgt[order]
    first = np.ones(len(order), dtype=bool)
    first[1:] = tgt_sorted[1:] != tgt_sorted[:-1]
    win_src = idx[order][first]
    win_tgt = tgt_sorted[first]
    right = np.full(H * W, np.nan)
    right[win_tgt] = left.ravel()[win_src].astype(np.float64)
    noc = np.zeros(H * W, dtype=bool)
    noc[win_src] = True
    return right.reshape(H, W), noc.reshape(H, W)


def gen_pair(H: int, W: int, n_cells: int, dmin: float, dmax: float, seed: int) -> StereoPair:
    """One rectified pair with planar-cell ground truth (left view is the reference)."""
    rng = _rng(seed)
    left = _quantise(_texture(rng, H, W))
    disp = _planar_cells(rng, H, W, n_cells, dmin, dmax)
    warped, noc = _forward_warp(left, disp)
    fill = _texture(rng, H, W)
    holes = np.isnan(warped)
    warped[holes] = fill[holes]
    right = _quantise(warped + rng.normal(0.0, 2.0, size=(H, W)))
    return StereoPair(left=left, right=right, gt=disp.astype(np.float32), noc=noc,
                      occ=np.ones((H, W), dtype=bool))


def gen_shift_pair(H: int, W: int, shift: int, seed: int) -> StereoPair:
    """Noise-free pair whose right view is the left view moved by a constant integer shift.

    right[y, x] = left[y, x + shift]; columns with no source take fresh texture.
    """
    rng = _rng(seed)
    left = _quantise(_texture(rng, H, W))
    fill = _quantise(_texture(rng, H, W))
    right = fill.copy()
    if shift < W:
        right[:, :W - shift] = left[:, shift:]
    gt = np.full((H, W), float(shift), dtype=np.float32)
    noc = np.zeros((H, W), dtype=bool)
    noc[:, shift:] = True
    return StereoPair(left=left, right=right, gt=gt, noc=noc, occ=np.ones((H, W), dtype=bool))


def gen_preset(name: str, index: int = 0) -> StereoPair:
    """Pair ``index`` of workload preset ``name`` (seed seed0 + index).  The
    uneven preset draws its 64 sizes (W = 8 U{80..160}, H = 8 U{24..48}) from
    seed 4999 and a disparity range of a quarter of the width."""
    c = PRESETS[name]
    seed = c["seed0"] + index
    if name == "uneven64":
        size_rng = _rng(4999)
        Ws = 8 * size_rng.integers(80, 161, size=64)
        Hs = 8 * size_rng.integers(24, 49, size=64)
        W, H = int(Ws[index]), int(Hs[index])
        d_low = int(np.rint(W / 16.0))
        D_full = 4 * d_low
        p = gen_pair(H, W, c["n_cells"], 0.0, float(D_full - 2), seed)
        p.D = d_low
        return p
    p = gen_pair(c["H"], c["W"], c["n_cells"], c["dmin"], c["dmax"], seed)
    p.D = c["D"]
    return p


def he_init_params(shapes, seed: int, bias_scale: float = 0.0):
    """He-normal weights for a list of conv shapes (out_ch, in_ch, k), drawn in list order.

    Weights are OIHW float32 with std sqrt(2 / (in_ch * k * k)).  Biases are zero
    unless ``bias_scale`` > 0, in which case they are U(-bias_scale, bias_scale),
    drawn after all weights.
    """
    rng = _rng(seed)
    ws = []
    for (o, i, k) in shapes:
        std = np.sqrt(2.0 / (i * k * k))
        ws.append((rng.standard_normal((o, i, k, k)) * std).astype(np.float32))
    bs = []
    for (o, i, k) in shapes:
        if bias_scale > 0:
            bs.append(rng.uniform(-bias_scale, bias_scale, size=o).astype(np.float32))
        else:
            bs.append(np.zeros(o, dtype=np.float32))
    return list(zip(ws, bs))


def gen_eps(shape, seed: int) -> np.ndarray:
    """Standard-normal reparameterisation noise, float32."""
    return _rng(seed).standard_normal(shape).astype(np.float32)
