"""GPU parity of the INT8 network (SV_I8) against the oracle's INT8 definition.

Integer sums are exact and every scale step is the same FP32 expression on
both sides, so the head's mu / logvar (which depend on every code decision
from E1 to the head) must match bit for bit; the refined map, whose last
layer is an FP32 MFMA projection, within 1e-5 normwise.  The distance from
the FP32 network is reported as an end-point error.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import quant, vae
from synth import gen_preset
from tests.gpu_util import cuda, flat_params, normwise, vae_params

pytestmark = pytest.mark.gpu


def _gpu(C, L, f, dtype, params, disp, img, H, W):
    import paper_2305_11566_amd as sv
    ref = sv.Refiner(*C, L, f, dtype)
    ref.pack(cuda(flat_params(params)))
    out, ml = ref.forward(cuda(disp), cuda(img), H, W)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ml.cpu().numpy()


def _compare(C, L, f, H, W, disp, img, seed=7):
    params = vae_params(C, L, seed)
    t = quant.forward(params, disp, img, f, H, W)
    out, ml = _gpu(C, L, f, "i8", params, disp, img, H, W)
    mu = ml[..., :L].transpose(0, 3, 1, 2)
    lv = ml[..., L:].transpose(0, 3, 1, 2)
    bad = int(np.sum(mu != t["mu"]) + np.sum(lv != t["logvar"]))
    assert bad == 0, f"{bad} mu/logvar values differ from the INT8 definition"
    e = normwise(out, t["out"])
    assert e <= 1e-5, f"out normwise {e:.3e}"
    return out, t, params


def test_i8_256x128():
    p = gen_preset("pair256x128")
    lo, _, _, d = oracle.match(p.left, p.right, 2, 5, 5, 16)
    _compare((16, 32, 64), 64, 2, 128, 256, d, lo)


def test_i8_1242x375_full_size():
    p = gen_preset("pair1242x375")
    lo, _, _, d = oracle.match(p.left, p.right, 4, 9, 7, 48)
    _compare((32, 64, 128), 128, 4, 375, 1242, d, lo)


@pytest.mark.parametrize("H,W,f,C,L,B", [
    (45, 63, 4, (8, 16, 24), 16, 2),     # odd sizes, every level ragged
    (8, 8, 8, (16, 16, 16), 8, 3),       # coarse map 1x1
    (100, 140, 2, (24, 40, 56), 32, 2),  # channel counts not multiples of 16
    (64, 512, 4, (32, 64, 128), 128, 1), # wide
])
def test_i8_shapes(H, W, f, C, L, B):
    rng = np.random.default_rng(H + W)
    h, w = -(-H // f), -(-W // f)
    disp = rng.integers(0, 40, (B, h, w)).astype(np.uint8)
    img = rng.integers(0, 256, (B, h, w)).astype(np.uint8)
    _compare(C, L, f, H, W, disp, img, seed=H)


def test_i8_zero_input_maps():
    # all-zero coarse maps: x0's amax is 0, every code is 0 and the scales 0
    C, L, f, H, W = (8, 16, 16), 8, 2, 20, 36
    z = np.zeros((1, 10, 18), np.uint8)
    _compare(C, L, f, H, W, z, z)


def test_i8_tile_shapes_bitwise_identical():
    import paper_2305_11566_amd as sv
    C, L, f, H, W = (16, 32, 64), 64, 2, 70, 90
    rng = np.random.default_rng(3)
    disp = rng.integers(0, 30, (2, 35, 45)).astype(np.uint8)
    img = rng.integers(0, 256, (2, 35, 45)).astype(np.uint8)
    params = vae_params(C, L, 5)
    base, bml = _gpu(C, L, f, "i8", params, disp, img, H, W)
    try:
        for cfg in (0, 1, 2, 3, 4, 6, 7, 9, 10, 11, 12, 13, 14, 15, 16 + 7, 48 + 2):
            for layer in range(9):
                sv.sv_set_layer_cfg(layer, cfg)
            out, ml = _gpu(C, L, f, "i8", params, disp, img, H, W)
            assert np.array_equal(ml, bml), sv.sv_conv_cfg_name(cfg)
            assert np.array_equal(out, base), sv.sv_conv_cfg_name(cfg)
    finally:
        for layer in range(9):
            sv.sv_set_layer_cfg(layer, -1)


def test_i8_epe_against_fp32():
    p = gen_preset("pair256x128")
    lo, _, _, d = oracle.match(p.left, p.right, 2, 5, 5, 16)
    C, L = (16, 32, 64), 64
    params = vae_params(C, L, 7)
    t64 = vae.forward(params, d, lo, 2, 128, 256)
    o8, _ = _gpu(C, L, 2, "i8", params, d, lo, 128, 256)
    o32, _ = _gpu(C, L, 2, "f32", params, d, lo, 128, 256)
    R = np.mean(np.abs(t64["out"] - 256.0 * t64["base"]))
    epe = float(np.mean(np.abs(o8 - o32)))
    print(f"i8 vs f32: mean EPE {epe:.4f} px, max {np.max(np.abs(o8 - o32)):.3f} px, mean |R| {R:.2f} px")
    assert epe <= 0.1 * R
