"""The per-frame path (census of both views, cost + WTA, network forward) as
the benchmark runs it: captured once in a HIP graph and replayed.  Every
replay, with eager work and synchronisations between replays, must give the
eager result bit for bit.  Also the profiling contract of the fused latent
kernel: an inference pass records it as the head's stage and nothing as G3's."""
import numpy as np
import pytest
import torch

from synth import gen_preset
from tests.gpu_util import cuda, flat_params, vae_params

pytestmark = pytest.mark.gpu

F, WW, WH, D = 4, 9, 7, 48
C, L = (32, 64, 128), 128


def _path(dtype, left, right, H, W):
    import paper_2305_11566_amd as sv
    B = left.shape[0]
    h, w = -(-H // F), -(-W // F)
    h3, w3 = h, w
    for _ in range(3):
        h3, w3 = -(-h3 // 2), -(-w3 // 2)
    dev = left.device
    bufs = {
        "cl": torch.empty((B, h, w), dtype=torch.int64, device=dev),
        "cr": torch.empty((B, h, w), dtype=torch.int64, device=dev),
        "low": torch.empty((B, h, w), dtype=torch.uint8, device=dev),
        "disp": torch.empty((B, h, w), dtype=torch.uint8, device=dev),
        "out": torch.empty((B, H, W), dtype=torch.float32, device=dev),
        "ml": torch.empty((B, h3, w3, 2 * L), dtype=torch.float32, device=dev),
    }
    ref = sv.Refiner(*C, L, F, dtype)
    ref.pack(cuda(flat_params(vae_params(C, L, 31))))
    ref.workspace(B, H, W)

    def step():
        sv.sv_census_pair(left, right, F, WW, WH, out=(bufs["cl"], bufs["cr"], bufs["low"]))
        sv.sv_cost_wta(bufs["cl"], bufs["cr"], D, WW * WH - 1, out=bufs["disp"])
        ref.forward(bufs["disp"], bufs["low"], H, W, out=bufs["out"], mu_logvar=bufs["ml"])
    return step, bufs


@pytest.mark.parametrize("e3name", [None, "th4_tn16_s2"])  # default; E3 split in two (its sum left to the fused kernel)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_graph_replays_equal_eager(dtype, e3name):
    import paper_2305_11566_amd as sv
    names = [sv.sv_conv_cfg_name(c) for c in range(sv.sv_num_layer_cfgs())]
    e3cfg = -1 if e3name is None else names.index(e3name)
    p = gen_preset("pair1242x375")
    H, W = p.left.shape
    left, right = cuda(p.left[None]), cuda(p.right[None])
    try:
        sv.sv_set_layer_cfg(2, e3cfg)
        step, bufs = _path(dtype, left, right, H, W)
        step()
        torch.cuda.synchronize()
        want = {k: v.clone() for k, v in bufs.items()}
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        for r in range(3):
            for v in bufs.values():  # eager work between replays
                v.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for k in ("cl", "cr", "low", "disp", "out", "ml"):
                assert torch.equal(bufs[k], want[k]), f"replay {r}: {k}"
            step()  # and an eager pass on the same buffers
            torch.cuda.synchronize()
            assert torch.equal(bufs["out"], want["out"])
        del g
    finally:
        sv.sv_set_layer_cfg(2, -1)


@pytest.mark.parametrize("fused", [True, False])
def test_profile_stages_of_the_latent_layers(fused):
    import paper_2305_11566_amd as sv
    p = gen_preset("pair256x128")
    H, W = p.left.shape
    left, right = cuda(p.left[None]), cuda(p.right[None])
    step, _ = _path("f32", left, right, H, W)
    try:
        sv.sv_set_latent_fusion(fused)
        step()
        torch.cuda.synchronize()
        sv.sv_profile_enable(4)
        for _ in range(2):
            step()
        prof = sv.sv_profile_read()
    finally:
        sv.sv_profile_enable(0)
        sv.sv_set_latent_fusion(True)
    assert prof["HEAD"][1] == 2 and prof["E3"][1] == 2 and prof["G2"][1] == 2
    assert prof["G3"][1] == (0 if fused else 2)
    assert prof["reparam"][1] == 0
