"""Pins of the oracle's Table I network (Sec. III-B1) and loss (Eqs. (9)-(11)).

The transposed convolution is pinned against torch's CPU float64
conv_transpose2d (a library special case), against the adjoint identity with
the separately pinned strided convolution, and by its impulse response.  The
whole network is pinned against an independent torch float64 composition
written here from Table I, plus closed forms: the last layer reduces to
linear interpolation for a tent kernel on X_0, and with zero weights the
head and the 1x1 deconvolution follow Eq. (8) in closed form.  The loss is
pinned by closed forms and central finite differences; the network's adjoint
against torch float64 autograd of the independent composition and against
central finite differences.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from oracle import tvae


def _rng(seed):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("k,s,H,W,extra", [(5, 2, 5, 7, 0), (5, 2, 5, 7, 1), (5, 2, 4, 3, 1),
                                           (3, 2, 6, 5, 1), (5, 4, 4, 6, 3), (5, 4, 3, 5, 0),
                                           (1, 1, 4, 5, 0), (5, 1, 6, 4, 0), (5, 3, 3, 4, 2)])
def test_tconv_matches_torch(k, s, H, W, extra):
    r = _rng(k * 100 + s * 10 + extra)
    B, C, O, pad = 2, 3, 4, (k - 1) // 2
    x = r.standard_normal((B, C, H, W))
    w = r.standard_normal((O, C, k, k))
    b = r.standard_normal(O)
    Ho = (H - 1) * s - 2 * pad + k + extra
    Wo = (W - 1) * s - 2 * pad + k + extra
    y = oracle.tconv2d(x, w, b, s, pad, Ho, Wo)
    ref = F.conv_transpose2d(torch.from_numpy(x), torch.from_numpy(w).transpose(0, 1).contiguous(),
                             torch.from_numpy(b), stride=s, padding=pad, output_padding=extra).numpy()
    assert y.shape == ref.shape
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("s,Ho,Wo", [(2, 9, 12), (2, 10, 11), (4, 15, 13), (1, 6, 5)])
def test_tconv_is_adjoint_of_strided_conv(s, Ho, Wo):
    # <tconv(x; W), y> = <x, conv(y; W^T)> when conv maps Ho x Wo back to x's size
    r = _rng(7 + s)
    k, pad, C, O = 5, 2, 3, 2
    H, W = (Ho + 2 * pad - k) // s + 1, (Wo + 2 * pad - k) // s + 1
    x = r.standard_normal((1, C, H, W))
    w = r.standard_normal((O, C, k, k))
    y = r.standard_normal((1, O, Ho, Wo))
    lhs = np.sum(oracle.tconv2d(x, w, None, s, pad, Ho, Wo) * y)
    rhs = np.sum(x * oracle.conv2d(y, np.ascontiguousarray(w.transpose(1, 0, 2, 3)), None, s, pad))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))


def test_tconv_impulse_response():
    k, s, pad = 5, 2, 2
    w = _rng(3).standard_normal((1, 1, k, k))
    x = np.zeros((1, 1, 4, 4))
    x[0, 0, 2, 1] = 1.0
    y = oracle.tconv2d(x, w, None, s, pad, 8, 8)
    exp = np.zeros((8, 8))
    for u in range(k):
        for v in range(k):
            Y, X = s * 2 + u - pad, s * 1 + v - pad
            if 0 <= Y < 8 and 0 <= X < 8:
                exp[Y, X] = w[0, 0, u, v]
    np.testing.assert_array_equal(y[0, 0], exp)


def _params(seed, scale=1.0):
    r = _rng(seed)
    out = []
    for (o, i, k) in tvae.layer_shapes():
        std = np.sqrt(2.0 / (i * k * k))
        out.append((scale * std * r.standard_normal((o, i, k, k)), 0.1 * r.standard_normal(o)))
    return out


def _torch_net(params, d, im, f, H, W, eps):
    """Table I written directly with torch float64 functional ops."""
    P = [(torch.from_numpy(np.asarray(w, np.float64)), torch.from_numpy(np.asarray(b, np.float64)))
         for (w, b) in params]
    (fe1, fe2, en1, en1r, en2, en2r, ms, d1, d1r, d2, d2r, dd, yy) = P
    act = lambda t: F.leaky_relu(t, 0.1)

    def conv(x, wb, s):
        return F.conv2d(x, wb[0], wb[1], stride=s, padding=(wb[0].shape[-1] - 1) // 2)

    def deconv(x, wb, s, size):
        k = wb[0].shape[-1]
        pad = (k - 1) // 2
        op = [size[i] - ((x.shape[2 + i] - 1) * s - 2 * pad + k) for i in range(2)]
        return F.conv_transpose2d(x, wb[0].transpose(0, 1), wb[1], stride=s, padding=pad,
                                  output_padding=tuple(op))

    x0 = torch.from_numpy(f * np.asarray(d, np.float64) / 256.0)[:, None]
    x1 = torch.from_numpy(np.asarray(im, np.float64) / 256.0)[:, None]
    FE1, FE2 = act(conv(x0, fe1, 1)), act(conv(x1, fe2, 1))
    E1 = act(conv(torch.cat([FE1, FE2], 1), en1, 2))
    E1R = act(conv(E1, en1r, 1))
    E2 = act(conv(torch.cat([E1, E1R], 1), en2, 2))
    E2R = act(conv(E2, en2r, 1))
    m = conv(torch.cat([E2, E2R], 1), ms, 1)
    z = (m[:, 0:1] - 1.0)
    if eps is not None:
        z = z + torch.from_numpy(eps) * torch.exp(m[:, 1:2] - 1.0)
    D1 = act(deconv(z, d1, 1, z.shape[2:]))
    D1R = act(conv(torch.cat([D1, E2, E2R], 1), d1r, 1))
    D2 = act(deconv(torch.cat([D1, E2, E2R, D1R], 1), d2, 2, E1.shape[2:]))
    D2R = act(conv(torch.cat([D2, E1, E1R], 1), d2r, 1))
    DD = act(deconv(torch.cat([D2, E1, E1R, D2R], 1), dd, 2, FE1.shape[2:]))
    Y = deconv(torch.cat([DD, x0, FE1, FE2], 1), yy, f, (H, W))[:, 0]
    return (256.0 * Y).numpy(), m.numpy()


def test_n_params():
    assert tvae.n_params() == 162380
    v = tvae.flatten(_params(1))
    assert v.size == tvae.n_params()
    back = tvae.unflatten(v)
    for (a, b), (c, d) in zip(_params(1), back):
        np.testing.assert_array_equal(a, c)
        np.testing.assert_array_equal(b, d)


@pytest.mark.parametrize("f,H,W,train", [(2, 32, 48, False), (2, 37, 53, True), (4, 45, 70, False),
                                         (4, 30, 81, True), (1, 13, 19, False)])
def test_forward_matches_torch(f, H, W, train):
    r = _rng(H * W + f)
    h, w = -(-H // f), -(-W // f)
    d = r.integers(0, 48, size=(2, h, w)).astype(np.uint8)
    im = r.integers(0, 256, size=(2, h, w)).astype(np.uint8)
    params = _params(11 + f)
    h3, w3 = -(-(-(-h // 2)) // 2), -(-(-(-w // 2)) // 2)
    eps = r.standard_normal((2, 1, h3, w3)) if train else None
    t = tvae.forward(params, d, im, f, H, W, eps)
    ref, ms = _torch_net(params, d, im, f, H, W, eps)
    assert t["out"].shape == (2, H, W)
    np.testing.assert_allclose(t["out"], ref, rtol=1e-10, atol=1e-9)
    np.testing.assert_allclose(t["mu"][:, 0], ms[:, 0], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(t["sigma"][:, 0], ms[:, 1], rtol=1e-10, atol=1e-12)


def test_final_layer_tent_kernel_is_linear_interpolation():
    # all weights zero except the final layer's on X_0 (input channel 16 of
    # "D & X_0 & FE_1 & FE_2"): a separable tent [0, 1/2, 1, 1/2, 0] with stride
    # 2 places X_0 on even outputs and the mean of neighbours on odd ones
    f, H, W = 2, 10, 14
    params = [(np.zeros((o, i, k, k)), np.zeros(o)) for (o, i, k) in tvae.layer_shapes()]
    tent = np.array([0.0, 0.5, 1.0, 0.5, 0.0])
    wy = np.zeros((1, 81, 5, 5))
    wy[0, 16] = np.outer(tent, tent)
    params[-1] = (wy, np.zeros(1))
    r = _rng(5)
    d = r.integers(0, 60, size=(1, H // 2, W // 2)).astype(np.uint8)
    im = r.integers(0, 256, size=(1, H // 2, W // 2)).astype(np.uint8)
    out = tvae.forward(params, d, im, f, H, W)["out"][0]
    x0 = f * d[0].astype(np.float64)  # full-res px

    def up(v):  # 1-D: even = sample, odd = mean with the next (0 past the end)
        n = v.shape[0]
        r_ = np.zeros((2 * n,) + v.shape[1:])
        r_[0::2] = v
        nxt = np.concatenate([v[1:], np.zeros((1,) + v.shape[1:])])
        r_[1::2] = 0.5 * (v + nxt)
        return r_

    exp = up(up(x0).T).T
    np.testing.assert_allclose(out, exp, rtol=0, atol=1e-12)


def test_head_and_first_deconv_follow_eq8():
    # zero weights up to D_1: mu and sigma are the head's biases everywhere and
    # D_1 = lrelu(w * z + b) with z = (mu - 1) + eps * exp(sigma - 1)
    params = [(np.zeros((o, i, k, k)), np.zeros(o)) for (o, i, k) in tvae.layer_shapes()]
    bmu, bsig = 0.7, 1.3
    params[tvae.NAMES.index("MS")] = (np.zeros((2, 48, 1, 1)), np.array([bmu, bsig]))
    wd1 = np.linspace(-1.0, 1.0, 32).reshape(32, 1, 1, 1)
    bd1 = np.linspace(0.2, -0.3, 32)
    params[tvae.NAMES.index("D_1")] = (wd1, bd1)
    r = _rng(9)
    d = r.integers(0, 30, size=(1, 12, 16)).astype(np.uint8)
    im = r.integers(0, 256, size=(1, 12, 16)).astype(np.uint8)
    eps = r.standard_normal((1, 1, 3, 4))
    t = tvae.forward(params, d, im, 2, 24, 32, eps)
    z = (bmu - 1.0) + eps[:, 0] * np.exp(bsig - 1.0)
    pre = wd1[:, 0, 0, 0][None, :, None, None] * z[:, None] + bd1[None, :, None, None]
    np.testing.assert_allclose(t["D_1"], np.where(pre > 0, pre, 0.1 * pre), rtol=1e-14, atol=1e-15)
    np.testing.assert_array_equal(t["mu"], np.full((1, 1, 3, 4), bmu))


def test_loss_closed_forms():
    r = _rng(2)
    B, H, W = 2, 6, 9
    gt = r.uniform(0, 100, size=(B, H, W))
    noc = r.random((B, H, W)) < 0.7
    occ = np.ones((B, H, W), bool)
    mu = np.ones((B, 1, 2, 3))
    sig = np.ones((B, 1, 2, 3))
    tot, l1, l2, *_ = tvae.loss(gt, gt, noc, occ, mu, sig)
    assert tot == 0.0 and l1 == 0.0 and l2 == 0.0
    # constant error e px: noc points count twice
    e = 1.75
    _, l1, _, *_ = tvae.loss(gt + e, gt, noc, occ, mu, sig)
    assert abs(l1 - e * (noc.sum() + occ.sum()) / occ.sum()) < 1e-12
    # mu = 1 + a: 256 * a^2 / 2; sigma = 1 + s: 256 * (e^{2s} - 1 - 2s) / 2
    a, s = 0.3, -0.4
    _, _, l2, *_ = tvae.loss(gt, gt, noc, occ, mu + a, sig)
    assert abs(l2 - 256.0 * 0.5 * a * a) < 1e-12
    _, _, l2, *_ = tvae.loss(gt, gt, noc, occ, mu, sig + s)
    assert abs(l2 - 256.0 * 0.5 * (np.exp(2 * s) - 1 - 2 * s)) < 1e-12


def test_loss_gradient_matches_finite_differences():
    r = _rng(4)
    B, H, W = 1, 5, 7
    gt = r.uniform(0, 50, size=(B, H, W))
    out = gt + r.uniform(0.5, 3.0, size=(B, H, W)) * r.choice([-1, 1], size=(B, H, W))
    noc = r.random((B, H, W)) < 0.6
    occ = r.random((B, H, W)) < 0.9
    occ |= noc
    mu = r.standard_normal((B, 1, 2, 2))
    sig = r.standard_normal((B, 1, 2, 2))
    _, _, _, dout, dmu, dsig = tvae.loss(out, gt, noc, occ, mu, sig)
    h = 1e-6
    for arr, grad in ((out, dout), (mu, dmu), (sig, dsig)):
        for idx in list(np.ndindex(arr.shape))[:12]:
            a = arr.copy()
            a[idx] += h
            args_p = [out, mu, sig]
            which = [out is arr, mu is arr, sig is arr].index(True)
            args_p[which] = a
            lp = tvae.loss(args_p[0], gt, noc, occ, args_p[1], args_p[2])[0]
            a = arr.copy()
            a[idx] -= h
            args_p[which] = a
            lm = tvae.loss(args_p[0], gt, noc, occ, args_p[1], args_p[2])[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, grad[idx])


@pytest.mark.parametrize("f,H,W,train", [(2, 24, 40, True), (4, 30, 45, False), (3, 19, 26, True)])
def test_backward_matches_torch_autograd(f, H, W, train):
    r = _rng(100 + f)
    h, w = -(-H // f), -(-W // f)
    d = r.integers(0, 40, size=(2, h, w)).astype(np.uint8)
    im = r.integers(0, 256, size=(2, h, w)).astype(np.uint8)
    params = _params(31 + f)
    h3, w3 = -(-(-(-h // 2)) // 2), -(-(-(-w // 2)) // 2)
    eps = r.standard_normal((2, 1, h3, w3)) if train else None
    dout = r.standard_normal((2, H, W))
    dmu = r.standard_normal((2, 1, h3, w3))
    dsg = r.standard_normal((2, 1, h3, w3))
    t = tvae.forward(params, d, im, f, H, W, eps)
    grads = tvae.backward(params, t, dout, dmu, dsg)
    # torch float64 autograd of the independent composition
    P = [(torch.tensor(np.asarray(w_), requires_grad=True), torch.tensor(np.asarray(b_), requires_grad=True))
         for (w_, b_) in params]
    import torch.nn.functional as Fn
    act = lambda z: Fn.leaky_relu(z, 0.1)

    def conv(x, wb, s):
        return Fn.conv2d(x, wb[0], wb[1], stride=s, padding=(wb[0].shape[-1] - 1) // 2)

    def deconv(x, wb, s, size):
        k = wb[0].shape[-1]
        pad = (k - 1) // 2
        op = [size[i] - ((x.shape[2 + i] - 1) * s - 2 * pad + k) for i in range(2)]
        return Fn.conv_transpose2d(x, wb[0].transpose(0, 1), wb[1], stride=s, padding=pad, output_padding=tuple(op))

    (fe1, fe2, en1, en1r, en2, en2r, ms, d1, d1r, d2, d2r, dd, yy) = P
    x0 = torch.from_numpy(f * d.astype(np.float64) / 256.0)[:, None]
    x1 = torch.from_numpy(im.astype(np.float64) / 256.0)[:, None]
    FE1, FE2 = act(conv(x0, fe1, 1)), act(conv(x1, fe2, 1))
    E1 = act(conv(torch.cat([FE1, FE2], 1), en1, 2)); E1R = act(conv(E1, en1r, 1))
    E2 = act(conv(torch.cat([E1, E1R], 1), en2, 2)); E2R = act(conv(E2, en2r, 1))
    m = conv(torch.cat([E2, E2R], 1), ms, 1)
    z = m[:, 0:1] - 1.0
    if eps is not None:
        z = z + torch.from_numpy(eps) * torch.exp(m[:, 1:2] - 1.0)
    D1 = act(deconv(z, d1, 1, z.shape[2:])); D1R = act(conv(torch.cat([D1, E2, E2R], 1), d1r, 1))
    D2 = act(deconv(torch.cat([D1, E2, E2R, D1R], 1), d2, 2, E1.shape[2:]))
    D2R = act(conv(torch.cat([D2, E1, E1R], 1), d2r, 1))
    DD = act(deconv(torch.cat([D2, E1, E1R, D2R], 1), dd, 2, FE1.shape[2:]))
    Y = deconv(torch.cat([DD, x0, FE1, FE2], 1), yy, f, (H, W))[:, 0]
    L = (torch.from_numpy(dout) * 256.0 * Y).sum() + (torch.from_numpy(dmu) * m[:, 0:1]).sum() \
        + (torch.from_numpy(dsg) * m[:, 1:2]).sum()
    L.backward()
    for name, (gw, gb), (tw, tb) in zip(tvae.NAMES, grads, P):
        np.testing.assert_allclose(gw, tw.grad.numpy(), rtol=1e-9, atol=1e-9 * max(1.0, np.abs(tw.grad.numpy()).max()),
                                   err_msg=name)
        np.testing.assert_allclose(gb, tb.grad.numpy(), rtol=1e-9, atol=1e-9 * max(1.0, np.abs(tb.grad.numpy()).max()),
                                   err_msg=name)


def test_backward_matches_finite_differences():
    # independent of torch: central differences of the same scalar on a tiny instance
    f, H, W = 2, 16, 24
    r = _rng(77)
    d = r.integers(0, 20, size=(1, 8, 12)).astype(np.uint8)
    im = r.integers(0, 256, size=(1, 8, 12)).astype(np.uint8)
    params = _params(5)
    eps = r.standard_normal((1, 1, 2, 3))
    dout = r.standard_normal((1, H, W))
    dmu = r.standard_normal((1, 1, 2, 3))
    dsg = r.standard_normal((1, 1, 2, 3))

    def scalar(ps):
        t = tvae.forward(ps, d, im, f, H, W, eps)
        return float(np.sum(dout * t["out"]) + np.sum(dmu * t["mu"]) + np.sum(dsg * t["sigma"])), t

    base, t = scalar(params)
    grads = tvae.backward(params, t, dout, dmu, dsg)
    checked = 0
    for li in range(len(params)):
        w, b = params[li]
        for idx in [tuple(r.integers(0, s) for s in w.shape) for _ in range(3)] + [None]:
            hh = 1e-6
            ps_p = [(a.copy(), c.copy()) for (a, c) in params]
            ps_m = [(a.copy(), c.copy()) for (a, c) in params]
            if idx is None:
                ps_p[li][1][0] += hh; ps_m[li][1][0] -= hh
                g = grads[li][1][0]
            else:
                ps_p[li][0][idx] += hh; ps_m[li][0][idx] -= hh
                g = grads[li][0][idx]
            lp, tp = scalar(ps_p)
            lm, tm = scalar(ps_m)
            # skip coordinates whose step flips a leaky-ReLU sign somewhere
            flips = any(np.any(np.sign(tp[k]) != np.sign(tm[k])) for k in tvae.NAMES[:-1] if k in tp and k != "MS")
            if flips:
                continue
            fd = (lp - lm) / (2 * hh)
            assert abs(fd - g) <= 1e-5 * max(1.0, abs(fd)), (tvae.NAMES[li], idx, fd, g)
            checked += 1
    assert checked >= 30
