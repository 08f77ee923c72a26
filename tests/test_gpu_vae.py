"""GPU parity of the refinement network's forward pass against the FP64 oracle.

FP32: normwise max|y - y64| / max|y64| <= 1e-5 on the refined disparity and on
mu / logvar.  BF16 / FP16: end-point error reported and bounded loosely (the
bar for reduced precision is an EPE statement, not bitwise parity).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import vae
from synth import gen_preset, gen_pair, gen_eps
from tests.gpu_util import cuda, flat_params, normwise, vae_params

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


def _inputs(H, W, f, ww, wh, D, seed, B=1):
    disp, img = [], []
    for b in range(B):
        p = gen_pair(H, W, 4, 1.0, max(2.0, f * D * 0.8), seed=seed + b)
        lo, _, _, d = oracle.match(p.left, p.right, f, ww, wh, D)
        disp.append(d[0]); img.append(lo[0])
    return np.stack(disp), np.stack(img)


def _gpu_forward(C, L, f, dtype, params, disp, img, H, W, eps=None):
    import paper_2305_11566_amd as sv
    ref = sv.Refiner(*C, L, f, dtype)
    ref.pack(cuda(flat_params(params)))
    saved = ref.saved_buffer(disp.shape[0], H, W) if eps is not None else None
    out, ml = ref.forward(cuda(disp), cuda(img), H, W, eps=None if eps is None else cuda(eps),
                          saved=saved)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ml.cpu().numpy()


def _compare(C, L, f, H, W, disp, img, seed=7, eps=None, dtype="f32", tol=TOL_F32):
    params = vae_params(C, L, seed)
    t = vae.forward(params, disp, img, f, H, W, eps=None if eps is None else eps.transpose(0, 3, 1, 2))
    out, ml = _gpu_forward(C, L, f, dtype, params, disp, img, H, W, eps)
    e_out = normwise(out, t["out"])
    mu = ml[..., :L].transpose(0, 3, 1, 2)
    lv = ml[..., L:].transpose(0, 3, 1, 2)
    e_ml = max(normwise(mu, t["mu"]), normwise(lv, t["logvar"]))
    assert e_out <= tol, f"out normwise {e_out:.3e}"
    assert e_ml <= tol, f"mu/logvar normwise {e_ml:.3e}"
    return e_out, out, t


def test_f32_256x128():
    p = gen_preset("pair256x128")
    lo, _, _, d = oracle.match(p.left, p.right, 2, 5, 5, 16)
    _compare((16, 32, 64), 64, 2, 128, 256, d, lo)


def test_f32_1242x375_full_size():
    p = gen_preset("pair1242x375")
    lo, _, _, d = oracle.match(p.left, p.right, 4, 9, 7, 48)
    _compare((32, 64, 128), 128, 4, 375, 1242, d, lo)


@pytest.mark.parametrize("H,W,f,C,L,B", [
    (45, 63, 4, (8, 16, 24), 16, 2),     # odd sizes, every level ragged
    (18, 18, 2, (8, 8, 8), 8, 1),        # coarsest level 2x2 -> 1x1 ... small
    (8, 8, 8, (16, 16, 16), 8, 3),       # coarse map 1x1: all levels 1x1
    (100, 140, 2, (24, 40, 56), 32, 2),  # channel counts not multiples of 16
    (64, 512, 4, (32, 64, 128), 128, 1), # wide
])
def test_f32_shapes(H, W, f, C, L, B):
    rng = np.random.default_rng(H + W)
    h, w = -(-H // f), -(-W // f)
    disp = rng.integers(0, 40, (B, h, w)).astype(np.uint8)
    img = rng.integers(0, 256, (B, h, w)).astype(np.uint8)
    _compare(C, L, f, H, W, disp, img, seed=H)


def test_f32_training_forward_with_eps():
    p = gen_preset("pair256x128")
    lo, _, _, d = oracle.match(p.left, p.right, 2, 5, 5, 16)
    eps = gen_eps((1, 8, 16, 64), seed=9000)
    _compare((16, 32, 64), 64, 2, 128, 256, d, lo, eps=eps)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_reduced_precision_epe(dtype):
    """Mean end-point error against the FP64 oracle, in full-res px, on He-init
    weights (a refinement term of about 50 px, so a stress case: the 0.05 px
    bar applies to the realistic refinement of the precision workload
    below)."""
    p = gen_preset("pair256x128")
    lo, _, _, d = oracle.match(p.left, p.right, 2, 5, 5, 16)
    params = vae_params((16, 32, 64), 64, 7)
    t = vae.forward(params, d, lo, 2, 128, 256)
    out, _ = _gpu_forward((16, 32, 64), 64, 2, dtype, params, d, lo, 128, 256)
    epe = float(np.mean(np.abs(out - t["out"])))
    scale = float(np.mean(np.abs(t["out"])))
    print(f"{dtype}: mean EPE {epe:.4f} px, max {np.max(np.abs(out - t['out'])):.3f} px, mean |out| {scale:.2f}")
    # measured 0.15 px (BF16) and 0.018 px (FP16); about 1.7x of headroom
    assert epe <= {"bf16": 0.25, "f16": 0.03}[dtype]


def _precision_params(C, L, seed, f_scale):
    """He-init weights with the final layer scaled by f_scale: 0.01 gives a
    refinement term of a few px, as trained weights do, where He-init's is
    of order 100 px."""
    params = vae_params(C, L, seed)
    wF, bF = params[8]
    params[8] = ((wF * np.float32(f_scale)).astype(np.float32), (bF * np.float32(f_scale)).astype(np.float32))
    return params


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_precision_bar_batch8_256x128(dtype):
    """The 8-pair 256x128 precision workload (seeds 3000-3007) through census
    + WTA and the 256x128 network with the final layer at 0.01 x He-init:
    mean |out - out_f32| <= 0.05 px, and the same bar against the FP64
    oracle."""
    import paper_2305_11566_amd as sv
    C, L, f, H, W, D = (16, 32, 64), 64, 2, 128, 256, 16
    ps = [gen_preset("batch8_256x128", i) for i in range(8)]
    left = cuda(np.stack([p.left for p in ps]))
    right = cuda(np.stack([p.right for p in ps]))
    cl, cr, low = sv.sv_census_pair(left, right, f, 5, 5)
    disp = sv.sv_cost_wta(cl, cr, D, 24)
    torch.cuda.synchronize()
    d_np, lo_np = disp.cpu().numpy(), low.cpu().numpy()
    ref_d = [oracle.match(p.left, p.right, f, 5, 5, D) for p in ps]
    assert np.array_equal(d_np, np.concatenate([r[3] for r in ref_d]))
    params = _precision_params(C, L, 7003, 0.01)
    t = vae.forward(params, d_np, lo_np, f, H, W)
    o32, _ = _gpu_forward(C, L, f, "f32", params, d_np, lo_np, H, W)
    o16, _ = _gpu_forward(C, L, f, dtype, params, d_np, lo_np, H, W)
    gt = np.stack([p.gt for p in ps])
    vs32 = np.abs(o16.astype(np.float64) - o32)
    vs64 = np.abs(o16 - t["out"])
    print(f"{dtype} 8x256x128: vs f32 mean {vs32.mean():.4f} max {vs32.max():.4f} px; vs oracle mean "
          f"{vs64.mean():.4f} max {vs64.max():.4f}; refinement term mean "
          f"{np.mean(np.abs(t['out'] - 256 * t['base'])):.3f} px; f32 vs gt {np.mean(np.abs(o32 - gt)):.3f}")
    assert normwise(o32, t["out"]) <= TOL_F32
    assert vs32.mean() <= 0.05
    assert vs64.mean() <= 0.05


def _split_of(name):
    return int(name.rsplit("_s", 1)[1]) if "_s" in name else 1


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_tile_configs_bitwise_identical(dtype):
    """Every tile shape gives the same bits; a split channel reduction gives
    the same bits for every tile shape at that split, and differs from the
    unsplit result only by rounding."""
    import paper_2305_11566_amd as sv
    rng = np.random.default_rng(5)
    C, L, f, H, W = (32, 64, 128), 128, 4, 150, 330
    h, w = -(-H // f), -(-W // f)
    disp = rng.integers(0, 48, (2, h, w)).astype(np.uint8)
    img = rng.integers(0, 256, (2, h, w)).astype(np.uint8)
    params = vae_params(C, L, 11)
    base, _ = _gpu_forward(C, L, f, dtype, params, disp, img, H, W)
    per_split = {1: base}
    tol = 1e-5 if dtype == "f32" else 1e-2
    try:
        for cfg in range(sv.sv_num_layer_cfgs()):
            for layer in range(9):
                sv.sv_set_layer_cfg(layer, cfg)
            out, _ = _gpu_forward(C, L, f, dtype, params, disp, img, H, W)
            name = sv.sv_conv_cfg_name(cfg)
            sp = _split_of(name)
            if sp not in per_split:
                per_split[sp] = out
                err = normwise(out, base)
                assert err <= tol, f"{name}: split result {err:.2e} from the unsplit one"
            assert (out == per_split[sp]).all(), f"cfg {cfg} ({name})"
    finally:
        for layer in range(9):
            sv.sv_set_layer_cfg(layer, -1)
    assert sorted(per_split) == [1, 2, 3, 4]


@pytest.mark.parametrize("e3name", [None, "th4_tn16_s2", "th4_tn16_s4"])  # E3 default, split in 2, in 4 (capped)
@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("C,L,f,H,W,B", [
    ((32, 64, 128), 128, 4, 375, 1242, 1),  # full size: 468 latent pixels, a tail of 4 past 16s
    ((32, 64, 128), 128, 4, 375, 1242, 9),  # 4212 latent pixels: one workgroup per 16 pixels (not two roles)
    ((16, 32, 64), 64, 2, 128, 256, 2),     # 256x128 widths, two images
    ((32, 64, 96), 32, 2, 50, 90, 3),       # 96 / 32 channels, 7x12 latent grids
    ((16, 24, 48), 16, 2, 30, 40, 1),       # FP32 fused; L = 16 is not a whole 16-bit chunk: two launches
])
def test_fused_latent_bitwise_equals_two_launches(dtype, C, L, f, H, W, B, e3name):
    """Inference runs the head and G3 as one kernel: same bits as the two
    layers launched one by one, unsplit (their configurations pinned to an
    unsplit tile shape).  When E3 runs split, the fused kernel also adds E3's
    partial sums in place of the second pass."""
    import paper_2305_11566_amd as sv
    rng = np.random.default_rng(H + W + B)
    h, w = -(-H // f), -(-W // f)
    disp = rng.integers(0, 40, (B, h, w)).astype(np.uint8)
    img = rng.integers(0, 256, (B, h, w)).astype(np.uint8)
    params = vae_params(C, L, 21)
    names = [sv.sv_conv_cfg_name(c) for c in range(sv.sv_num_layer_cfgs())]
    e3cfg = -1 if e3name is None else names.index(e3name)
    th4_tn16 = names.index("th4_tn16")
    try:
        for layer in (3, 4):
            sv.sv_set_layer_cfg(layer, th4_tn16)  # no split
        sv.sv_set_layer_cfg(2, e3cfg)
        sv.sv_set_latent_fusion(True)
        a, ma = _gpu_forward(C, L, f, dtype, params, disp, img, H, W)
        sv.sv_set_latent_fusion(False)
        b, mb = _gpu_forward(C, L, f, dtype, params, disp, img, H, W)
    finally:
        sv.sv_set_latent_fusion(True)
        for layer in (2, 3, 4):
            sv.sv_set_layer_cfg(layer, -1)
    assert np.array_equal(ma, mb), "mu / logvar"
    assert np.array_equal(a, b), "refined map"


def test_split_reduction_against_oracle():
    """Every layer forced to a 2-, 3- and 4-way channel split: FP32 forward
    within 1e-5 normwise of the oracle at the paper-sized shape."""
    import paper_2305_11566_amd as sv
    names = [sv.sv_conv_cfg_name(c) for c in range(sv.sv_num_layer_cfgs())]
    p = gen_preset("pair1242x375")
    lo, _, _, d = oracle.match(p.left, p.right, 4, 9, 7, 48)
    params = vae_params((32, 64, 128), 128, 7002)
    t = vae.forward(params, d, lo, 4, 375, 1242)
    try:
        for sp in (2, 3, 4):
            cfg = names.index(f"th4_tn16_s{sp}")
            for layer in range(9):
                sv.sv_set_layer_cfg(layer, cfg)
            out, _ = _gpu_forward((32, 64, 128), 128, 4, "f32", params, d, lo, 375, 1242)
            err = normwise(out, t["out"])
            assert err <= 1e-5, f"split {sp}: {err:.2e}"
    finally:
        for layer in range(9):
            sv.sv_set_layer_cfg(layer, -1)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_many_tile_batch_equals_single_images(dtype):
    """Three full-size images in one call (1,440 tiles of the final gather,
    spread over the XCDs in another order than one image's 480) give the same
    bits as three single-image calls, with every layer on the same unsplit
    tile shape; FP32 also within 1e-5 of the oracle."""
    import paper_2305_11566_amd as sv
    C, L, f, H, W, B = (32, 64, 128), 128, 4, 375, 1242, 3
    disp, img = _inputs(H, W, f, 9, 7, 48, seed=7100, B=B)
    params = vae_params(C, L, 7002)
    names = [sv.sv_conv_cfg_name(c) for c in range(sv.sv_num_layer_cfgs())]
    th4_tn16 = names.index("th4_tn16")
    try:
        for layer in range(1, 8):
            sv.sv_set_layer_cfg(layer, th4_tn16)
        a, ma = _gpu_forward(C, L, f, dtype, params, disp, img, H, W)
        for b in range(B):
            o, m = _gpu_forward(C, L, f, dtype, params, disp[b:b + 1], img[b:b + 1], H, W)
            assert np.array_equal(m[0], ma[b]), f"image {b}: mu / logvar"
            assert np.array_equal(o[0], a[b]), f"image {b}: refined map"
    finally:
        for layer in range(1, 8):
            sv.sv_set_layer_cfg(layer, -1)
    if dtype == "f32":
        t = vae.forward(params, disp, img, f, H, W)
        assert normwise(a, t["out"]) <= TOL_F32
