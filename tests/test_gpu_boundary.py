"""The binding's argument checks and the batch call's host behaviour.

Buffers of the wrong shape, dtype or device are refused with ValueError /
TypeError before any library call (the C ABI sees only pointers, so a short
buffer would be read or written past on the device); none of these cases
launches a kernel.  sv_stereo_batch returns without waiting for the device:
two calls made while the stream is still busy with earlier work come back
before that work ends, and their results equal those of calls on an idle
stream.
"""
import time

import numpy as np
import pytest
import torch

import paper_2305_11566_amd as sv
from synth import gen_pair
from tests.gpu_util import cuda, flat_params, vae_params

pytestmark = pytest.mark.gpu

C, L, F, WW, WH = (32, 64, 128), 128, 4, 9, 7


def test_matching_outputs_of_the_wrong_shape_are_refused():
    img = torch.zeros((2, 40, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        sv.sv_census(img, 4, 9, 7, out=(torch.empty((2, 10, 15), dtype=torch.int64, device="cuda"), None))
    with pytest.raises(TypeError):
        sv.sv_census(img, 4, 9, 7, out=(torch.empty((2, 10, 16), dtype=torch.int32, device="cuda"), None))
    cl = torch.zeros((2, 10, 16), dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):
        sv.sv_census_pair(img, img, 4, 9, 7, out=(cl, cl.clone(), torch.empty((2, 10, 15), dtype=torch.uint8,
                                                                             device="cuda")))
    with pytest.raises(ValueError):
        sv.sv_cost_wta(cl, cl, 8, 62, out=torch.empty((2, 10, 15), dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError):
        sv.sv_sgm(cl, cl, 8, 62, 10, 120, workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    low = torch.zeros((2, 10, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        sv.sv_zncc_cost(low, low[:, :9], 8, 9, 7)
    with pytest.raises(ValueError):
        sv.sv_smp_median(low, 8, out=torch.empty((2, 10, 17), dtype=torch.uint8, device="cuda"))


def test_network_buffers_of_the_wrong_shape_are_refused():
    ref = sv.Refiner(*C, L, F, "f32")
    H, W = 40, 64
    d = torch.zeros((1, 10, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):   # coarse map of a 36-row pair passed for 40 rows
        ref.forward(torch.zeros((1, 9, 16), dtype=torch.uint8, device="cuda"), d[:, :9], H, W)
    with pytest.raises(ValueError):
        ref.forward(d, d, H, W, out=torch.empty((1, H, W - 1), device="cuda"))
    with pytest.raises(ValueError):
        ref.forward(d, d, H, W, mu_logvar=torch.empty((1, 2, 2, L), device="cuda"))
    with pytest.raises(ValueError):
        ref.forward(d, d, H, W, eps=torch.empty((1, 2, 2, L - 1), device="cuda"),
                    saved=ref.saved_buffer(1, H, W))
    with pytest.raises(ValueError):
        ref.forward(d, d, H, W, eps=torch.empty((1, 2, 2, L), device="cuda"),
                    saved=torch.empty(64, dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError):
        ref.backward(ref.saved_buffer(1, H, W), 1, H, W, None, torch.empty((1, H, W + 1), device="cuda"), 1e-3)
    with pytest.raises(ValueError):
        sv.sv_loss(torch.empty((1, H, W), device="cuda"), torch.empty((1, H, W - 1), device="cuda"), None, L, 1e-3)
    t = sv.TableVAE(F, "f32")
    with pytest.raises(ValueError):
        t.forward(d[:, :9], d[:, :9], H, W)
    plan = sv.BatchPlan(*C, L, F, "f32", 2, 64, 64, 8, WW, WH)
    l = torch.zeros((40, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        plan.run([(l, l[:39], 4)], ref.packed)
    with pytest.raises(ValueError):
        plan.run([(l, l, 4)], ref.packed, outs=[torch.empty((40, 63), device="cuda")])
    with pytest.raises(ValueError):
        plan.run([(l, l, 4)], ref.packed, disp_outs=[torch.empty((10, 15), dtype=torch.uint8, device="cuda")])
    plan.close()


def test_stereo_batch_returns_without_waiting_for_the_device():
    params = vae_params(C, L, seed=19)
    ref = sv.Refiner(*C, L, F, "bf16")
    ref.pack(cuda(flat_params(params)))
    sizes = [(96, 200, 12), (120, 320, 20), (37, 61, 8)]
    pairs = []
    for i, (H, W, D) in enumerate(sizes):
        p = gen_pair(H, W, 5, 0.0, float(4 * D - 2), seed=950 + i)
        pairs.append((cuda(p.left), cuda(p.right), D))
    plan = sv.BatchPlan(*C, L, F, "bf16", 4, 128, 320, 32, WW, WH)
    idle = [o.clone() for o in plan.run(pairs, ref.packed)]      # graph captured, idle stream
    idle2 = [o.clone() for o in plan.run(pairs[::-1], ref.packed)]
    torch.cuda.synchronize()
    # keep the stream busy for a while (a bounded spin), then call twice
    done = torch.cuda.Event()
    torch.cuda._sleep(200_000_000)
    t0 = time.perf_counter()
    a = plan.run(pairs, ref.packed)
    b = plan.run(pairs[::-1], ref.packed)
    t_calls = time.perf_counter() - t0
    done.record()
    busy = not done.query()
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    print(f"two calls returned after {t_calls * 1e3:.2f} ms; stream drained after {t_all * 1e3:.1f} ms")
    assert busy, "the stream was idle before the calls returned: the spin was too short to tell"
    assert t_calls < 0.5 * t_all
    for x, y in zip(a, idle):
        assert torch.equal(x, y)
    for x, y in zip(b, idle2):
        assert torch.equal(x, y)
    plan.close()
