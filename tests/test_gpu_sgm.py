"""GPU parity of semi-global matching (Eqs. (4)-(6)) and of the single matching
phase + median (Eq. (7)): bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from synth import gen_preset, gen_pair
from tests.gpu_util import bits, cuda

pytestmark = pytest.mark.gpu


def _gpu(cl, cr, D, nbits, P1, P2):
    import paper_2305_11566_amd as sv
    tl = cuda(cl.view(np.int64))
    tr = cuda(cr.view(np.int64))
    raw = sv.sv_sgm(tl, tr, D, nbits, P1, P2)
    post = sv.sv_smp_median(raw, D)
    torch.cuda.synchronize()
    return raw.cpu().numpy(), post.cpu().numpy()


def _check(cl, cr, D, nbits, P1, P2):
    raw, post = _gpu(cl, cr, D, nbits, P1, P2)
    ref_raw = oracle.wta(oracle.sgm(oracle.cost_volume(cl, cr, D, nbits), P1, P2))
    assert (raw == ref_raw).all(), f"SGM disparity: {np.sum(raw != ref_raw)} of {raw.size} differ"
    ref_post = oracle.median3(oracle.smp(ref_raw, D))
    assert (post == ref_post).all(), f"SMP + median: {np.sum(post != ref_post)} of {post.size} differ"
    return raw, post


def _census_pair(left, right, f, ww, wh):
    lo_l, lo_r = oracle.downsample(left, f), oracle.downsample(right, f)
    return oracle.census(lo_l, ww, wh), oracle.census(lo_r, ww, wh)


@pytest.mark.parametrize("k", ["pair256x128", "pair1242x375"])
def test_workload_pairs(k):
    p = gen_preset(k)
    f, ww, wh, D = {"pair256x128": (2, 5, 5, 16), "pair1242x375": (4, 9, 7, 48)}[k]
    cl, cr = _census_pair(p.left[None], p.right[None], f, ww, wh)
    _check(cl, cr, D, ww * wh - 1, 10, 120)


def test_uneven_batch_pairs_wide_ranges():
    # the 64-pair workload's ranges reach 80 (two and more disparities per lane)
    for i in (0, 7, 63):
        p = gen_preset("uneven64", i)
        cl, cr = _census_pair(p.left[None], p.right[None], 4, 9, 7)
        _check(cl, cr, p.D, 62, 10, 120)


@pytest.mark.parametrize("h,w,D,P1,P2", [
    (1, 1, 1, 10, 120),       # single pixel
    (7, 5, 16, 10, 120),      # w < D
    (3, 300, 256, 10, 120),   # D = 256: 16 disparities per lane
    (9, 40, 33, 10, 120),     # ragged lane split
    (12, 17, 8, 0, 0),        # zero penalties: plain winner-take-all
    (5, 70, 64, 1, 2),
    (40, 1, 4, 3, 9),         # one column
])
def test_edge_shapes(h, w, D, P1, P2):
    rng = np.random.default_rng(h * 100 + w)
    cl = rng.integers(0, 2 ** 62, (2, h, w), dtype=np.uint64)
    cr = np.roll(cl, 2, axis=2) ^ rng.integers(0, 2 ** 3, (2, h, w), dtype=np.uint64)
    raw, _ = _check(cl, cr, D, 62, P1, P2)
    if P1 == 0 and P2 == 0:
        assert (raw == oracle.wta(oracle.cost_volume(cl, cr, D, 62))).all()


def test_sgm_then_network_runs_and_is_deterministic():
    import paper_2305_11566_amd as sv
    p = gen_preset("pair1242x375")
    l, r = cuda(p.left[None]), cuda(p.right[None])
    cl, cr, low = sv.sv_census_pair(l, r, 4, 9, 7)
    a = sv.sv_smp_median(sv.sv_sgm(cl, cr, 48, 62, 10, 120), 48)
    b = sv.sv_smp_median(sv.sv_sgm(cl, cr, 48, 62, 10, 120), 48)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("k", ["pair256x128", "pair1242x375"])
def test_zncc_cost_and_sgm_workload_pairs(k):
    import paper_2305_11566_amd as sv
    p = gen_preset(k)
    f, ww, wh, D = {"pair256x128": (2, 5, 5, 16), "pair1242x375": (4, 9, 7, 48)}[k]
    lo_l, lo_r = oracle.downsample(p.left[None], f), oracle.downsample(p.right[None], f)
    tl, tr = cuda(lo_l), cuda(lo_r)
    c = sv.sv_zncc_cost(tl, tr, D, ww, wh)
    raw = sv.sv_zncc_sgm(tl, tr, D, ww, wh, 10, 120)
    post = sv.sv_smp_median(raw, D)
    torch.cuda.synchronize()
    ref_c = oracle.zncc_cost(lo_l, lo_r, D, ww, wh)
    assert (c.cpu().numpy().astype(np.int32) == ref_c).all(), \
        f"ZNCC cost: {np.sum(c.cpu().numpy() != ref_c)} of {ref_c.size} differ"
    ref_raw = oracle.wta(oracle.sgm(ref_c, 10, 120))
    assert (raw.cpu().numpy() == ref_raw).all()
    assert (post.cpu().numpy() == oracle.median3(oracle.smp(ref_raw, D))).all()


@pytest.mark.parametrize("h,w,D,ww,wh", [(1, 1, 1, 3, 3), (6, 9, 12, 5, 3), (20, 70, 64, 9, 9),
                                          (5, 300, 256, 7, 7), (33, 17, 20, 3, 5)])
def test_zncc_edge_shapes(h, w, D, ww, wh):
    import paper_2305_11566_amd as sv
    rng = np.random.default_rng(h * 7 + w)
    ll = rng.integers(0, 256, (2, h, w), dtype=np.uint8)
    lr = np.roll(ll, 2, axis=2) ^ rng.integers(0, 3, (2, h, w), dtype=np.uint8)
    ll[0, : max(1, h // 2), : max(1, w // 3)] = 40    # flat windows
    c = sv.sv_zncc_cost(cuda(ll), cuda(lr), D, ww, wh)
    torch.cuda.synchronize()
    assert (c.cpu().numpy().astype(np.int32) == oracle.zncc_cost(ll, lr, D, ww, wh)).all()


def test_zncc_unsupported_window_is_an_error():
    import paper_2305_11566_amd as sv
    ll = cuda(np.zeros((1, 8, 8), np.uint8))
    with pytest.raises(sv.SvError):
        sv.sv_zncc_cost(ll, ll, 4, 11, 3)
