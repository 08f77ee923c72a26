"""GPU parity of sv_paper_batch, the paper's whole system (reduction, ZNCC +
SGM or census + SGM, single matching phase + median, Table I network) on
pairs of uneven sizes: bitwise equal to the per-pair calls, the coarse maps
bit-exact and the FP32 outputs within 1e-5 normwise of the oracle, and a
captured graph's replays equal to the eager call."""
import numpy as np
import pytest
import torch

import oracle
from oracle import tvae
from synth import gen_pair, gen_preset, he_init_params
from tests.gpu_util import cuda, flat_params, normwise

pytestmark = pytest.mark.gpu

P1, P2 = 10, 120


def _net(dtype, f, seed=31):
    import paper_2305_11566_amd as sv
    params = he_init_params(tvae.layer_shapes(), seed=seed, bias_scale=0.1)
    net = sv.TableVAE(f, dtype)
    net.pack(cuda(flat_params(params)))
    return net, params


def _pairs(kind):
    if kind == "uneven64":
        ps = [gen_preset("uneven64", i) for i in (3, 17, 40)]
        return [(p.left, p.right, p.D) for p in ps], 4, 9, 7
    sizes = [(96, 160, 12), (75, 203, 16), (128, 256, 16)]
    out = []
    for k, (H, W, D) in enumerate(sizes):
        p = gen_pair(H, W, 6, 4.0, 24.0, seed=6100 + k)
        out.append((p.left, p.right, D))
    return out, 2, 5, 5


def _per_pair(net, matcher, median, f, ww, wh, left, right, D):
    """The same steps through the single-purpose calls."""
    import paper_2305_11566_amd as sv
    l, r = cuda(left[None]), cuda(right[None])
    cl, cr, low = sv.sv_census_pair(l, r, f, ww, wh)
    _, low_r = sv.sv_census(r, f, ww, wh)
    if matcher == "zncc":
        disp = sv.sv_zncc_sgm(low, low_r, D, ww, wh, P1, P2)
    else:
        disp = sv.sv_sgm(cl, cr, D, ww * wh - 1, P1, P2)
    if median:
        disp = sv.sv_smp_median(disp, D)
    out, _ = net.forward(disp, low, left.shape[0], left.shape[1])
    return out[0], disp[0]


@pytest.mark.parametrize("matcher,median,dtype,kind", [
    ("zncc", True, "f32", "small"), ("zncc", True, "bf16", "uneven64"), ("census", True, "f32", "uneven64"),
    ("census", False, "bf16", "small"), ("zncc", False, "f16", "small"),
])
def test_paper_batch_equals_per_pair_calls(matcher, median, dtype, kind):
    import paper_2305_11566_amd as sv
    pairs, f, ww, wh = _pairs(kind)
    net, _ = _net(dtype, f)
    maxH = max(p[0].shape[0] for p in pairs)
    maxW = max(p[0].shape[1] for p in pairs)
    maxD = max(p[2] for p in pairs)
    pb = sv.PaperBatch(matcher, f, ww, wh, P1, P2, dtype, median, maxH, maxW, maxD)
    tp = [(cuda(l), cuda(r), D) for l, r, D in pairs]
    disp_outs = [torch.empty((-(-l.shape[0] // f), -(-l.shape[1] // f)), dtype=torch.uint8, device="cuda")
                 for l, _, _ in pairs]
    outs = pb.run(tp, net.packed, disp_outs=disp_outs)
    torch.cuda.synchronize()
    for (l, r, D), o, dl in zip(pairs, outs, disp_outs):
        ref_out, ref_disp = _per_pair(net, matcher, median, f, ww, wh, l, r, D)
        torch.cuda.synchronize()
        assert torch.equal(dl, ref_disp), f"{l.shape}: coarse map"
        assert torch.equal(o.view(torch.int32), ref_out.view(torch.int32)), f"{l.shape}: refined map"


def test_paper_batch_f32_against_oracle():
    """ZNCC + SGM + SMP + median + Table I network (FP32) on three pairs of
    different sizes: coarse maps bit-exact with the oracle, refined maps within
    1e-5 normwise of the FP64 network."""
    import paper_2305_11566_amd as sv
    pairs, f, ww, wh = _pairs("small")
    net, params = _net("f32", f)
    pb = sv.PaperBatch("zncc", f, ww, wh, P1, P2, "f32", True, 128, 256, 16)
    tp = [(cuda(l), cuda(r), D) for l, r, D in pairs]
    disp_outs = [torch.empty((-(-l.shape[0] // f), -(-l.shape[1] // f)), dtype=torch.uint8, device="cuda")
                 for l, _, _ in pairs]
    outs = pb.run(tp, net.packed, disp_outs=disp_outs)
    torch.cuda.synchronize()
    for (l, r, D), o, dl in zip(pairs, outs, disp_outs):
        H, W = l.shape
        lo, _, d = oracle.match_zncc_sgm(l[None], r[None], f, ww, wh, D, P1, P2)
        assert np.array_equal(dl.cpu().numpy(), d[0]), f"{W}x{H}: coarse map"
        t = tvae.forward(params, d, lo, f, H, W)
        e = normwise(o.cpu().numpy()[None], t["out"])
        assert e <= 1e-5, f"{W}x{H}: normwise {e:.2e}"


def test_paper_batch_graph_replays_equal_eager():
    import paper_2305_11566_amd as sv
    pairs, f, ww, wh = _pairs("small")
    net, _ = _net("bf16", f)
    pb = sv.PaperBatch("zncc", f, ww, wh, P1, P2, "bf16", True, 128, 256, 16)
    tp = [(cuda(l), cuda(r), D) for l, r, D in pairs]
    eager = [o.clone() for o in pb.run(tp, net.packed)]
    torch.cuda.synchronize()
    outs = [torch.empty_like(o) for o in eager]
    g = torch.cuda.CUDAGraph()
    pb.run(tp, net.packed, outs=outs)  # warm-up outside the capture
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        pb.run(tp, net.packed, outs=outs)
    for _ in range(3):
        for o in outs:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o.view(torch.int32), e.view(torch.int32))
