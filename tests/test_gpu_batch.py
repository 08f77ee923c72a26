"""Batches of uneven pairs through one graph replay: bitwise equal to the
per-pair calls, the FP32 result within tolerance of the oracle, graph replay
equal to eager launches, and the autotuner (which may only change speed)."""
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import vae
from synth import gen_preset, gen_pair
from tests.gpu_util import cuda, flat_params, normwise, vae_params

pytestmark = pytest.mark.gpu

C, L, F, WW, WH = (32, 64, 128), 128, 4, 9, 7


def _per_pair(ref, left, right, D):
    import paper_2305_11566_amd as sv
    cl, cr, low = sv.sv_census_pair(left[None], right[None], F, WW, WH)
    disp = sv.sv_cost_wta(cl, cr, D, WW * WH - 1)
    out, _ = ref.forward(disp, low, left.shape[0], left.shape[1])
    return out[0], disp[0]


def _pairs(sizes, seed0):
    out = []
    for i, (H, W, D) in enumerate(sizes):
        p = gen_pair(H, W, 5, 0.0, float(4 * D - 2), seed=seed0 + i)
        out.append((cuda(p.left), cuda(p.right), D))
    return out


SIZES = [(96, 200, 12), (37, 61, 8), (120, 320, 20), (64, 64, 16), (8, 8, 1), (75, 250, 30)]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batch_equals_per_pair_bitwise(dtype):
    import paper_2305_11566_amd as sv
    params = vae_params(C, L, seed=13)
    ref = sv.Refiner(*C, L, F, dtype)
    ref.pack(cuda(flat_params(params)))
    pairs = _pairs(SIZES, 600)
    plan = sv.BatchPlan(*C, L, F, dtype, 8, 128, 320, 32, WW, WH)
    disp_outs = [torch.empty((-(-H // F), -(-W // F)), dtype=torch.uint8, device="cuda")
                 for (H, W, _) in SIZES]
    outs = plan.run(pairs, ref.packed, disp_outs=disp_outs)
    torch.cuda.synchronize()
    for (l, r, D), o, d in zip(pairs, outs, disp_outs):
        po, pd = _per_pair(ref, l, r, D)
        torch.cuda.synchronize()
        assert torch.equal(pd, d)
        assert torch.equal(po, o)
    plan.close()


def test_batch_f32_against_oracle():
    import paper_2305_11566_amd as sv
    params = vae_params(C, L, seed=14)
    ref = sv.Refiner(*C, L, F, "f32")
    ref.pack(cuda(flat_params(params)))
    sizes = [(120, 320, 20), (75, 250, 30)]
    pairs = _pairs(sizes, 700)
    plan = sv.BatchPlan(*C, L, F, "f32", 4, 128, 320, 32, WW, WH)
    outs = plan.run(pairs, ref.packed)
    torch.cuda.synchronize()
    for (H, W, D), (l, r, _), o in zip(sizes, pairs, outs):
        lo, _, _, d = oracle.match(l.cpu().numpy(), r.cpu().numpy(), F, WW, WH, D)
        t = vae.forward(params, d, lo, F, H, W)
        assert normwise(o.cpu().numpy()[None], t["out"]) <= 1e-5
    plan.close()


# pairs of the 64-pair uneven workload: the widest (1280x256), the largest
# (1152x384), the smallest (640x200) and every eighth
UNEVEN_IDX = [1, 2, 29, 0, 8, 16, 24, 40, 56]


def test_uneven_workload_f32_against_oracle():
    """FP32 batch at the uneven workload's real sizes (widths 640-1280,
    heights 200-384, D 40-80): coarse maps bit-exact with the oracle's
    census + WTA, refined maps within 1e-5 normwise of the FP64 network."""
    import paper_2305_11566_amd as sv
    params = vae_params(C, L, seed=18)
    ref = sv.Refiner(*C, L, F, "f32")
    ref.pack(cuda(flat_params(params)))
    ps = [gen_preset("uneven64", i) for i in UNEVEN_IDX]
    pairs = [(cuda(p.left), cuda(p.right), p.D) for p in ps]
    disp_outs = [torch.empty((-(-p.left.shape[0] // F), -(-p.left.shape[1] // F)), dtype=torch.uint8,
                             device="cuda") for p in ps]
    plan = sv.BatchPlan(*C, L, F, "f32", 64, 384, 1280, 80, WW, WH)
    outs = plan.run(pairs, ref.packed, disp_outs=disp_outs)
    torch.cuda.synchronize()
    for i, p, o, dg in zip(UNEVEN_IDX, ps, outs, disp_outs):
        H, W = p.left.shape
        lo, _, _, d = oracle.match(p.left, p.right, F, WW, WH, p.D)
        assert np.array_equal(dg.cpu().numpy(), d[0]), f"pair {i} ({W}x{H}, D {p.D}): coarse map"
        t = vae.forward(params, d, lo, F, H, W)
        e = normwise(o.cpu().numpy()[None], t["out"])
        assert e <= 1e-5, f"pair {i} ({W}x{H}): normwise {e:.2e}"
    plan.close()


def test_uneven_workload_pairs_subset():
    """Eight pairs of the 64-pair uneven workload (widths 640-1280, heights 192-384)."""
    import paper_2305_11566_amd as sv
    params = vae_params(C, L, seed=15)
    ref = sv.Refiner(*C, L, F, "bf16")
    ref.pack(cuda(flat_params(params)))
    ps = [gen_preset("uneven64", i) for i in range(0, 64, 8)]
    pairs = [(cuda(p.left), cuda(p.right), p.D) for p in ps]
    plan = sv.BatchPlan(*C, L, F, "bf16", 64, 384, 1280, 80, WW, WH)
    outs = plan.run(pairs, ref.packed)
    torch.cuda.synchronize()
    for (l, r, D), o in zip(pairs, outs):
        po, _ = _per_pair(ref, l, r, D)
        torch.cuda.synchronize()
        assert torch.equal(po, o)
    plan.close()


def test_graph_replays_equal_eager():
    """Several replays of the captured graph with different pair sets, eager
    work in between; each checked against the eager launches."""
    import paper_2305_11566_amd as sv
    params = vae_params(C, L, seed=16)
    ref = sv.Refiner(*C, L, F, "bf16")
    ref.pack(cuda(flat_params(params)))
    plan = sv.BatchPlan(*C, L, F, "bf16", 8, 128, 320, 32, WW, WH)
    sets = [SIZES[:3], SIZES[2:], SIZES[::2], SIZES]
    for k, sizes in enumerate(sets):
        pairs = _pairs(sizes, 800 + 10 * k)
        g = plan.run(pairs, ref.packed)
        torch.cuda.synchronize()
        os.environ["SV_DISABLE_GRAPH"] = "1"
        try:
            e = plan.run(pairs, ref.packed)
            torch.cuda.synchronize()
        finally:
            del os.environ["SV_DISABLE_GRAPH"]
        _ = torch.ones(1000, device="cuda").sum().item()   # unrelated eager work between replays
        for a, b in zip(g, e):
            assert torch.equal(a, b)
    plan.close()


def test_autotune_cache_and_results_unchanged(tmp_path, monkeypatch):
    import paper_2305_11566_amd as sv
    cache = tmp_path / "tune.tsv"
    monkeypatch.setenv("SV_AUTOTUNE_CACHE", str(cache))
    params = vae_params(C, L, seed=17)
    ref = sv.Refiner(*C, L, F, "bf16")
    ref.pack(cuda(flat_params(params)))
    pairs = _pairs(SIZES[:4], 900)
    plan = sv.BatchPlan(*C, L, F, "bf16", 8, 128, 320, 32, WW, WH)
    before = [o.clone() for o in plan.run(pairs, ref.packed)]
    plan.close()
    try:
        sv.sv_autotune(*C, L, F, "bf16", 2, 128, 320, 32, WW, WH)
        txt = cache.read_text()
        assert "128x320" in txt and len(txt.strip().split("\n")) == 1
        plan = sv.BatchPlan(*C, L, F, "bf16", 8, 128, 320, 32, WW, WH)
        after = plan.run(pairs, ref.packed)
        torch.cuda.synchronize()
        for a, b in zip(before, after):
            assert torch.equal(a, b)
        plan.close()
        # a corrupt cache is ignored with a warning
        cache.write_text("garbage line\n")
        plan = sv.BatchPlan(*C, L, F, "bf16", 8, 128, 320, 32, WW, WH)
        again = plan.run(pairs, ref.packed)
        torch.cuda.synchronize()
        for a, b in zip(before, again):
            assert torch.equal(a, b)
        plan.close()
    finally:
        for layer in range(9):
            sv.sv_set_layer_cfg(layer, -1)
        sv.sv_set_cost_wta_split(0)
