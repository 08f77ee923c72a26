"""sv_vae_forward_static (no workspace, no allocation) against sv_vae_forward:
two calls in a row, the second on a smaller input, each bitwise equal to the
workspace entry point on the same inputs; a shape beyond the fixed scratch is
refused before anything is enqueued."""
import numpy as np
import pytest
import torch

import oracle
from synth import gen_pair, gen_preset
from tests.gpu_util import cuda, flat_params, vae_params

pytestmark = pytest.mark.gpu

C, L, F = (32, 64, 128), 128, 4


def _coarse(H, W, seed, D=48):
    p = gen_pair(H, W, 6, 0.0, float(4 * D - 2), seed=seed)
    lo, _, _, d = oracle.match(p.left, p.right, F, 9, 7, D)
    return d, lo


@pytest.mark.parametrize("dtype", ["f32", "bf16", "i8"])
def test_static_scratch_equals_workspace_entry_point(dtype):
    import paper_2305_11566_amd as sv
    ref = sv.Refiner(*C, L, F, dtype)
    ref.pack(cuda(flat_params(vae_params(C, L, seed=31))))
    p = gen_preset("pair1242x375")
    lo, _, _, d = oracle.match(p.left, p.right, F, 9, 7, 48)
    cases = [(d, lo, 375, 1242)]
    d2, lo2 = _coarse(200, 320, seed=77, D=20)      # a smaller second input
    cases.append((d2, lo2, 200, 320))
    for dd, ll, H, W in cases:
        dt, lt = cuda(dd), cuda(ll)
        a, ma = ref.forward_static(dt, lt, H, W)
        b, mb = ref.forward(dt, lt, H, W)
        torch.cuda.synchronize()
        assert torch.equal(a, b), f"{dtype} {W}x{H}: refined map"
        assert torch.equal(ma, mb), f"{dtype} {W}x{H}: mu / logvar"


def test_static_scratch_refuses_shapes_beyond_it():
    import paper_2305_11566_amd as sv
    from paper_2305_11566_amd._lib import SvError
    ref = sv.Refiner(*C, L, F, "f32")
    ref.pack(cuda(flat_params(vae_params(C, L, seed=32))))
    B, H, W = 4, 375, 1242
    d = torch.zeros((B, 94, 311), dtype=torch.uint8, device="cuda")
    with pytest.raises(SvError) as e:
        ref.forward_static(d, d, H, W)
    assert e.value.status == -5   # SV_ERR_WORKSPACE
