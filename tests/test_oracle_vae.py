"""Pins of the oracle's FP64 network primitives, forward, loss, adjoint and Adam.

Library special cases (torch CPU float64 conv2d / interpolate / autograd, used
only here as independent checks), closed forms, dot-product (adjoint)
identities and central finite differences.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from oracle import vae
from synth import gen_pair, he_init_params, gen_eps


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


# ------------------------------------------------------------- conv / resize

@pytest.mark.parametrize("k,s", [(3, 1), (3, 2), (1, 1)])
def test_conv_matches_torch(k, s):
    x = _rand((2, 3, 9, 7), 1)
    w = _rand((4, 3, k, k), 2)
    b = _rand(4, 3)
    pad = (k - 1) // 2
    y = oracle.conv2d(x, w, b, s, pad)
    ref = F.conv2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b), stride=s, padding=pad)
    np.testing.assert_allclose(y, ref.numpy(), rtol=1e-12, atol=1e-12)


def test_conv_impulse_response_and_1x1_matmul():
    x = np.zeros((1, 1, 7, 7))
    x[0, 0, 3, 3] = 1.0
    w = _rand((2, 1, 3, 3), 4)
    y = oracle.conv2d(x, w, None, 1, 1)
    # a correlation of an impulse returns the kernel flipped around the impulse
    np.testing.assert_array_equal(y[0, :, 2:5, 2:5], w[:, 0, ::-1, ::-1])
    x = _rand((2, 5, 4, 3), 5)
    w = _rand((6, 5, 1, 1), 6)
    y = oracle.conv2d(x, w, None, 1, 0)
    np.testing.assert_allclose(y, np.einsum("oc,bchw->bohw", w[:, :, 0, 0], x), rtol=1e-13)


@pytest.mark.parametrize("hi,wi,ho,wo", [(5, 7, 10, 14), (94, 311, 375, 1242), (3, 4, 3, 4), (12, 39, 24, 78), (24, 78, 47, 156)])
def test_resize_matches_torch(hi, wi, ho, wo):
    x = _rand((2, hi, wi), 7)
    y = oracle.resize(x, ho, wo)
    ref = F.interpolate(torch.from_numpy(x)[:, None], size=(ho, wo), mode="bilinear", align_corners=False)
    np.testing.assert_allclose(y, ref[:, 0].numpy(), rtol=1e-12, atol=1e-12)


def test_resize_constant_identity_ramp():
    assert np.allclose(oracle.resize(np.full((1, 4, 5), 3.25), 9, 11), 3.25, rtol=0, atol=1e-15)
    x = _rand((1, 6, 8), 8)
    np.testing.assert_array_equal(oracle.resize(x, 6, 8), x)
    # an affine ramp a + b*x is reproduced exactly at output columns whose source
    # position falls inside [0, n_in - 1] (away from the clamped border)
    wi, wo = 8, 20
    ramp = np.tile(2.0 + 0.5 * np.arange(wi), (1, 3, 1))
    y = oracle.resize(ramp, 3, wo)
    s = (np.arange(wo) + 0.5) * wi / wo - 0.5
    inside = (s >= 0) & (s <= wi - 1)
    np.testing.assert_allclose(y[0, 1, inside], 2.0 + 0.5 * s[inside], rtol=1e-14)


@pytest.mark.parametrize("k,s,shape", [(3, 1, (2, 3, 9, 7)), (3, 2, (1, 4, 10, 9)), (1, 1, (2, 5, 3, 4))])
def test_conv_adjoints_dot_product(k, s, shape):
    """<conv(x), g> = <x, conv_dx(g)>  and  <conv_w(x), g> = <w, conv_dw(x, g)>."""
    x = _rand(shape, 9)
    w = _rand((6, shape[1], k, k), 10)
    pad = (k - 1) // 2
    y = oracle.conv2d(x, w, None, s, pad)
    g = _rand(y.shape, 11)
    dx = oracle.conv2d_dx(g, w, x.shape, s, pad)
    assert np.isclose(np.sum(y * g), np.sum(x * dx), rtol=1e-12)
    dw, db = oracle.conv2d_dw(x, g, k, s, pad)
    assert np.isclose(np.sum(y * g), np.sum(w * dw), rtol=1e-12)
    np.testing.assert_allclose(db, g.sum(axis=(0, 2, 3)), rtol=1e-12)


def test_resize_adjoint_dot_product():
    x = _rand((3, 5, 7), 12)
    y = oracle.resize(x, 13, 19)
    g = _rand(y.shape, 13)
    assert np.isclose(np.sum(y * g), np.sum(x * oracle.resize_adj(g, 5, 7)), rtol=1e-12)
    # downscaling direction too
    y = oracle.resize(x, 3, 4)
    g = _rand(y.shape, 14)
    assert np.isclose(np.sum(y * g), np.sum(x * oracle.resize_adj(g, 5, 7)), rtol=1e-12)


# ------------------------------------------------------------------ network

def _small_problem(seed=0, H=32, W=16, f=2, C=(4, 6, 8), L=5, bias_scale=0.1):
    pair = gen_pair(H, W, 3, 1.0, 6.0, seed=100 + seed)
    rng = np.random.default_rng(seed)
    h, w = -(-H // f), -(-W // f)
    disp = rng.integers(0, 8, (2, h, w)).astype(np.uint8)
    img = rng.integers(0, 256, (2, h, w)).astype(np.uint8)
    shapes = [(o, i, k) for (o, i, k, s) in vae.layer_shapes(*C, L)]
    params = he_init_params(shapes, seed=200 + seed, bias_scale=bias_scale)
    return pair, disp, img, params


class TorchNet:
    """Independent torch float64 composition of the network, for cross-checks only."""

    def __init__(self, params, f):
        self.p = [(torch.tensor(w, dtype=torch.float64, requires_grad=True),
                   torch.tensor(b, dtype=torch.float64, requires_grad=True)) for w, b in params]
        self.f = f

    def __call__(self, disp, img, H, W, eps=None):
        lr = lambda t: F.leaky_relu(t, 0.1)
        x0 = torch.stack([self.f * torch.tensor(disp, dtype=torch.float64) / 256.0,
                          torch.tensor(img, dtype=torch.float64) / 256.0], 1)
        conv = lambda x, i, s: F.conv2d(x, self.p[i][0], self.p[i][1], stride=s,
                                        padding=(self.p[i][0].shape[-1] - 1) // 2)
        up = lambda x, ref: F.interpolate(x, size=ref.shape[-2:], mode="bilinear", align_corners=False)
        e1 = lr(conv(x0, 0, 2))
        e2 = lr(conv(e1, 1, 2))
        e3 = lr(conv(e2, 2, 2))
        ml = conv(e3, 3, 1)
        L = ml.shape[1] // 2
        mu, lv = ml[:, :L], ml[:, L:]
        z = mu if eps is None else mu + torch.tensor(eps, dtype=torch.float64) * torch.exp(0.5 * lv)
        g3 = lr(conv(z, 4, 1))
        g2 = lr(conv(torch.cat([up(g3, e2), e2], 1), 5, 1))
        g1 = lr(conv(torch.cat([up(g2, e1), e1], 1), 6, 1))
        g0 = lr(conv(torch.cat([up(g1, x0), x0], 1), 7, 1))
        catf = F.interpolate(torch.cat([g0, x0], 1), size=(H, W), mode="bilinear", align_corners=False)
        r = conv(catf, 8, 1)[:, 0]
        base = F.interpolate(x0[:, :1], size=(H, W), mode="bilinear", align_corners=False)[:, 0]
        return 256.0 * (base + r), mu, lv


def test_forward_matches_torch_composition():
    pair, disp, img, params = _small_problem(seed=1, H=40, W=28, f=2)
    t = vae.forward(params, disp, img, 2, 40, 28)
    out, mu, lv = TorchNet(params, 2)(disp, img, 40, 28)
    np.testing.assert_allclose(t["out"], out.detach().numpy(), rtol=1e-11, atol=1e-9)
    np.testing.assert_allclose(t["mu"], mu.detach().numpy(), rtol=1e-11, atol=1e-12)


def test_forward_odd_sizes_factor4():
    pair, disp, img, params = _small_problem(seed=2, H=45, W=63, f=4)
    t = vae.forward(params, disp, img, 4, 45, 63)
    out, _, _ = TorchNet(params, 4)(disp, img, 45, 63)
    assert t["x0"].shape[-2:] == (12, 16)
    np.testing.assert_allclose(t["out"], out.detach().numpy(), rtol=1e-11, atol=1e-9)


def test_zero_final_weights_reduce_to_linear_upscaling():
    """All-zero final-layer weights: R is its bias, so the output is the linear
    upscaling of the coarse map plus a constant (the paper's Mini+Linear)."""
    pair, disp, img, params = _small_problem(seed=3, H=32, W=48, f=2)
    wF, bF = params[8]
    params[8] = (np.zeros_like(wF), np.array([0.125], np.float32))
    t = vae.forward(params, disp, img, 2, 32, 48)
    lin = oracle.resize(2.0 * disp.astype(np.float64), 32, 48)   # f*d in full-res px
    np.testing.assert_allclose(t["out"], lin + 256.0 * 0.125, rtol=1e-14, atol=1e-12)


def test_kl_and_smooth_l1_closed_forms():
    assert vae.kl_divergence(np.zeros((1, 3, 2, 2)), np.zeros((1, 3, 2, 2))) == 0.0
    # constant mu = 2, logvar = 0:  0.5 * 4 = 2
    assert np.isclose(vae.kl_divergence(np.full((1, 2, 3, 3), 2.0), np.zeros((1, 2, 3, 3))), 2.0)
    # mu = 0, logvar = log 3: 0.5 * (3 - 1 - log 3)
    assert np.isclose(vae.kl_divergence(np.zeros((1, 1, 2, 2)), np.full((1, 1, 2, 2), np.log(3.0))),
                      0.5 * (2.0 - np.log(3.0)))
    out = np.array([[0.0, 0.5, 3.0, -2.0]])
    gt = np.zeros_like(out)
    l, g = vae.smooth_l1(out, gt)
    assert np.isclose(l, (0.0 + 0.125 + 2.5 + 1.5) / 4)
    np.testing.assert_allclose(g, np.array([[0.0, 0.5, 1.0, -1.0]]) / 4)


def _total_loss(params, disp, img, f, H, W, eps, gt, klw):
    t = vae.forward(params, disp, img, f, H, W, eps)
    return vae.loss(t, gt, klw)[0], t


def test_backward_matches_torch_autograd():
    pair, disp, img, params = _small_problem(seed=4, H=32, W=16, f=2)
    L = params[3][0].shape[0] // 2
    t0 = vae.forward(params, disp, img, 2, 32, 16)
    eps = gen_eps(t0["mu"].shape, seed=9001)
    gt = np.stack([pair.gt, pair.gt[::-1]])
    klw = 0.3
    t = vae.forward(params, disp, img, 2, 32, 16, eps)
    total, data, kl, dout = vae.loss(t, gt, klw)
    grads = vae.backward(params, t, dout, klw)
    net = TorchNet(params, 2)
    out, mu, lv = net(disp, img, 32, 16, eps)
    e = out - torch.tensor(gt, dtype=torch.float64)
    data_t = F.smooth_l1_loss(out, torch.tensor(gt, dtype=torch.float64), beta=1.0)
    kl_t = torch.mean(0.5 * (mu ** 2 + torch.exp(lv) - 1.0 - lv))
    (data_t + klw * kl_t).backward()
    assert np.isclose(total, float((data_t + klw * kl_t).detach()), rtol=1e-12)
    for (dw, db), (tw, tb) in zip(grads, net.p):
        np.testing.assert_allclose(dw, tw.grad.numpy(), rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(db, tb.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_backward_finite_differences():
    """Central differences on the 32x16 instance, sampled weights of every layer
    plus every bias; coordinates whose +-h step crosses a kink are skipped."""
    pair, disp, img, params = _small_problem(seed=5, H=32, W=16, f=2)
    t0 = vae.forward(params, disp, img, 2, 32, 16)
    eps = gen_eps(t0["mu"].shape, seed=9002)
    gt = np.stack([pair.gt, pair.gt])
    klw = 0.5
    params64 = [(w.astype(np.float64), b.astype(np.float64)) for w, b in params]
    total, t = _total_loss(params64, disp, img, 2, 32, 16, eps, gt, klw)
    _, _, _, dout = vae.loss(t, gt, klw)
    grads = vae.backward(params64, t, dout, klw)
    rng = np.random.default_rng(77)
    checked = 0
    for li, (w, b) in enumerate(params64):
        coords = [("w", tuple(rng.integers(0, n) for n in w.shape)) for _ in range(32)]
        coords += [("b", (o,)) for o in range(min(b.size, 8))]
        for kind, idx in coords:
            arr = w if kind == "w" else b
            h = 1e-5 * max(1.0, abs(arr[idx]))
            vals = []
            kinks = []
            for sgn in (+1, -1):
                p2 = [(ww.copy(), bb.copy()) for ww, bb in params64]
                tgt = p2[li][0] if kind == "w" else p2[li][1]
                tgt[idx] += sgn * h
                l, tt = _total_loss(p2, disp, img, 2, 32, 16, eps, gt, klw)
                vals.append(l)
                kinks.append(tt)
            # skip if any pre-activation or smooth-L1 residual changes branch
            crossed = False
            for key in ("E1pre", "E2pre", "E3pre", "G3pre", "G2pre", "G1pre", "G0pre"):
                if np.any((kinks[0][key] > 0) != (kinks[1][key] > 0)):
                    crossed = True
            e0 = np.abs(kinks[0]["out"] - gt) < 1.0
            e1 = np.abs(kinks[1]["out"] - gt) < 1.0
            if crossed or np.any(e0 != e1):
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            an = grads[li][0][idx] if kind == "w" else grads[li][1][idx]
            # relative 1e-6, plus the rounding bound of a central difference
            roundoff = 8 * np.finfo(np.float64).eps * abs(total) / h
            assert abs(fd - an) <= 1e-6 * abs(an) + roundoff, (li, kind, idx, fd, an)
            checked += 1
    assert checked >= 200


def test_adam_first_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2, so the update is
    lr * g / (|g| + eps)."""
    rng = np.random.default_rng(12)
    w = rng.standard_normal(50)
    g = rng.standard_normal(50)
    w1, m, v = vae.adam_step(w, g, np.zeros(50), np.zeros(50), 1)
    np.testing.assert_allclose(w1, w - 5e-4 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.01 * g, rtol=1e-12)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)
    # constant gradient: m_hat stays g and v_hat stays g^2 at every step
    m = np.zeros(50); v = np.zeros(50); ww = w.copy()
    for s in range(1, 6):
        ww, m, v = vae.adam_step(ww, g, m, v, s)
    np.testing.assert_allclose(ww, w - 5 * 5e-4 * g / (np.abs(g) + 1e-8), rtol=1e-10)


def test_param_count_of_workload_shapes():
    assert vae.n_params(16, 32, 64, 64) == 73299
    assert vae.n_params(32, 64, 128, 128) == 290963
