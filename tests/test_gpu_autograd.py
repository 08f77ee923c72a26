"""autograd.Function over the kernels, the training loop and checkpoint/resume."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from oracle import vae
from synth import gen_pair, gen_eps
from tests.gpu_util import cuda, flat_params, normwise, vae_params

pytestmark = pytest.mark.gpu


def test_autograd_function_matches_oracle():
    """Loss written in torch (smooth-L1 + KL on the mu/logvar output): the
    gradient reaching the parameters equals the oracle's."""
    import paper_2305_11566_amd as sv
    from paper_2305_11566_amd.autograd import SvRefine
    H, W, f, C, L, B = 64, 96, 2, (8, 16, 24), 16, 2
    ps = [gen_pair(H, W, 3, 2.0, 12.0, seed=300 + b) for b in range(B)]
    m = [oracle.match(p.left, p.right, f, 5, 5, 8) for p in ps]
    disp = np.concatenate([x[3] for x in m]); img = np.concatenate([x[0] for x in m])
    gt = np.stack([p.gt for p in ps]).astype(np.float64)
    params = vae_params(C, L, seed=21)
    eps = gen_eps((B, 4, 6, L), seed=9300)
    klw = 0.1
    t = vae.forward(params, disp, img, f, H, W, eps=eps.transpose(0, 3, 1, 2))
    _, _, _, dref = vae.loss(t, gt, klw)
    g_or = vae.flatten(vae.backward(params, t, dref, klw))

    ref = sv.Refiner(*C, L, f, "f32")
    w = cuda(flat_params(params)).requires_grad_(True)
    out, ml = SvRefine.apply(w, ref, cuda(disp), cuda(img), H, W, cuda(eps))
    mu, lv = ml[..., :L], ml[..., L:]
    loss = F.smooth_l1_loss(out, cuda(gt.astype(np.float32)), beta=1.0) + \
        klw * torch.mean(0.5 * (mu ** 2 + torch.exp(lv) - 1.0 - lv))
    loss.backward()
    torch.cuda.synchronize()
    assert normwise(w.grad.cpu().numpy(), g_or) <= 1e-4


def _tiny_trainer(dtype="bf16"):
    from paper_2305_11566_amd.train import Trainer, layer_shapes
    from synth import he_init_params
    C, L = (16, 32, 64), 64
    p = he_init_params(layer_shapes(*C, L), seed=7005)
    flat = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in p])
    return Trainer(flat, C=C, latent=L, dtype=dtype)


def test_checkpoint_resume_bitwise(tmp_path):
    from paper_2305_11566_amd.train import make_pool, batch_indices
    left, right, gt = make_pool(8, 64, 128, seed0=5000)
    a = _tiny_trainer()
    for _ in range(6):
        idx = batch_indices(a.step, 4, 8).cuda()
        a.train_step(left[idx], right[idx], gt[idx])
    b = _tiny_trainer()
    for _ in range(3):
        idx = batch_indices(b.step, 4, 8).cuda()
        b.train_step(left[idx], right[idx], gt[idx])
    b.save(tmp_path / "ck.npz")
    c = _tiny_trainer()
    c.load(tmp_path / "ck.npz")
    for _ in range(3):
        idx = batch_indices(c.step, 4, 8).cuda()
        c.train_step(left[idx], right[idx], gt[idx])
    torch.cuda.synchronize()
    assert c.step == a.step == 6
    assert torch.equal(a.w, c.w) and torch.equal(a.m, c.m) and torch.equal(a.v, c.v)


def test_training_reduces_loss():
    from paper_2305_11566_amd.train import make_pool, batch_indices
    left, right, gt = make_pool(16, 64, 128, seed0=5000)
    tr = _tiny_trainer()
    first = None
    losses = []
    for _ in range(60):
        idx = batch_indices(tr.step, 8, 16).cuda()
        l = tr.train_step(left[idx], right[idx], gt[idx]).cpu().numpy().copy()
        losses.append(float(l[1]))
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:5]), losses[::10]
