"""GPU parity of reduction + census and Hamming cost + WTA: bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from synth import gen_preset, gen_pair
from tests.gpu_util import bits, cuda

pytestmark = pytest.mark.gpu


def _run_gpu(left, right, f, ww, wh, D):
    import paper_2305_11566_amd as sv
    l, r = cuda(left), cuda(right)
    cl, cr, low = sv.sv_census_pair(l, r, f, ww, wh)
    cl1, low1 = sv.sv_census(l, f, ww, wh)
    disp = sv.sv_cost_wta(cl, cr, D, ww * wh - 1)
    torch.cuda.synchronize()
    assert (bits(cl1) == bits(cl)).all() and (low1.cpu() == low.cpu()).all()
    return bits(cl), bits(cr), low.cpu().numpy(), disp.cpu().numpy()


def _check(left, right, f, ww, wh, D):
    if left.ndim == 2:
        left, right = left[None], right[None]
    gl, gr, glow, gd = _run_gpu(left, right, f, ww, wh, D)
    lo, cl, cr, d = oracle.match(left, right, f, ww, wh, D)
    assert (glow == lo).all(), "reduced image"
    assert (gl == cl).all(), "census left"
    assert (gr == cr).all(), "census right"
    assert (gd == d).all(), f"disparity: {np.sum(gd != d)} of {d.size} differ"


@pytest.mark.parametrize("k", ["pair256x128", "pair1242x375"])
def test_workload_pairs(k):
    p = gen_preset(k)
    c = {"pair256x128": (2, 5, 5, 16), "pair1242x375": (4, 9, 7, 48)}[k]
    _check(p.left, p.right, *c)


def test_uneven_batch_pairs():
    for i in (0, 7, 63):
        p = gen_preset("uneven64", i)
        _check(p.left, p.right, 4, 9, 7, p.D)


@pytest.mark.parametrize("H,W,f,ww,wh,D", [
    (13, 9, 1, 3, 3, 4),        # tiny, f = 1
    (37, 61, 3, 5, 5, 30),      # w < D at the reduced size (21 < 30)
    (5, 7, 2, 9, 7, 8),         # image smaller than the window
    (1, 1, 1, 3, 3, 1),         # single pixel, D = 1
    (70, 1100, 4, 9, 7, 256),   # D = 256, maximum
    (33, 150, 2, 5, 13, 40),    # 64-bit codes (5 x 13 window)
    (45, 333, 4, 17, 3, 20),    # widest window
    (129, 257, 2, 5, 5, 16),    # ragged tails in both directions
])
def test_edge_shapes(H, W, f, ww, wh, D):
    rng = np.random.default_rng(H * 1000 + W)
    left = rng.integers(0, 256, (2, H, W), dtype=np.uint8)
    right = np.roll(left, -3, axis=2) ^ rng.integers(0, 2, (2, H, W), dtype=np.uint8)
    _check(left, right, f, ww, wh, D)


@pytest.mark.parametrize("f", [1, 2, 3, 4, 5, 6, 7, 8])
def test_every_factor_ragged(f):
    # each reduction factor is its own kernel instantiation; sizes leave a
    # partial block in both directions
    H, W = 8 * f + f // 2 + 1, 64 * f + f - 1 if f > 1 else 131
    rng = np.random.default_rng(f)
    left = rng.integers(0, 256, (1, H, W), dtype=np.uint8)
    right = np.roll(left, -2 * f, axis=2) ^ rng.integers(0, 4, (1, H, W), dtype=np.uint8)
    _check(left, right, f, 7, 5, 12)


def test_tall_census_tiles():
    # enough tiles for the 16-row census tiles (two 1024x2048 views at f = 2)
    rng = np.random.default_rng(11)
    left = rng.integers(0, 256, (2, 1024, 2048), dtype=np.uint8)
    right = np.roll(left, -6, axis=2) ^ rng.integers(0, 4, (2, 1024, 2048), dtype=np.uint8)
    _check(left, right, 2, 9, 7, 24)


def test_identical_images_zero():
    p = gen_pair(96, 200, 4, 2.0, 20.0, seed=3)
    _, _, _, d = _run_gpu(p.left[None], p.left[None], 2, 5, 5, 16)
    assert (d == 0).all()


@pytest.mark.parametrize("dsplit", [1, 2, 4, 8])
def test_lane_split_variants_identical(dsplit):
    import paper_2305_11566_amd as sv
    p = gen_preset("pair1242x375")
    try:
        sv.sv_set_cost_wta_split(dsplit)
        _check(p.left, p.right, 4, 9, 7, 48)
    finally:
        sv.sv_set_cost_wta_split(0)


def test_determinism_repeat():
    p = gen_preset("pair1242x375")
    a = _run_gpu(p.left[None], p.right[None], 4, 9, 7, 48)
    b = _run_gpu(p.left[None], p.right[None], 4, 9, 7, 48)
    for x, y in zip(a, b):
        assert (x == y).all()


def test_large_batch_equals_single_images():
    """36 full-size pairs at f = 4 in one call (16-row census tiles, several
    rows per cost + WTA workgroup): every image's words, reduced image and
    disparities equal its single-image call (4-row tiles, one row per
    workgroup), and two of them equal the oracle."""
    import paper_2305_11566_amd as sv
    B = 36
    ps = [gen_pair(375, 1242, 5, 1.0, 150.0, seed=7300 + b) for b in range(B)]
    left = np.stack([p.left for p in ps])
    right = np.stack([p.right for p in ps])
    gl, gr, glow, gd = _run_gpu(left, right, 4, 9, 7, 48)
    for b in range(B):
        sl, sr, slow, sd = _run_gpu(left[b:b + 1], right[b:b + 1], 4, 9, 7, 48)
        assert (gl[b] == sl[0]).all() and (gr[b] == sr[0]).all(), f"image {b}: census"
        assert (glow[b] == slow[0]).all() and (gd[b] == sd[0]).all(), f"image {b}: reduced / disparity"
    for b in (0, B - 1):
        lo, cl, cr, d = oracle.match(left[b:b + 1], right[b:b + 1], 4, 9, 7, 48)
        assert (gl[b] == cl[0]).all() and (gr[b] == cr[0]).all() and (gd[b] == d[0]).all()
