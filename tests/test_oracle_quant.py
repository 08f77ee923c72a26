"""Pins of the oracle's INT8 network (quantised inference, Sec. V).

BF16 storage rounding is pinned against torch's bfloat16 conversion; the
quantiser by its closed-form properties; the integer convolution against the
separately pinned FP64 convolution of the dequantised codes; the FP32
bilinear resize bit for bit against its definition -- each weight the
correctly rounded FP32 value of the exact fractional source position
(derived here by integer arithmetic on the rational), the corners from the
half-pixel formula in exact arithmetic, the value from a scalar FP32 loop in
the stated order -- and loosely against the FP64 one; the whole pass by a
special case that reduces exactly to the FP network (bias-only weights) and
by a loose bound on its distance from the FP64 network.
"""
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
from oracle import quant, vae
from synth import he_init_params


def test_bf16_matches_torch_round_to_nearest_even():
    r = np.random.default_rng(0)
    x = (r.standard_normal(20000) * np.exp(r.uniform(-20, 20, 20000))).astype(np.float32)
    # exact ties between two BF16 neighbours, both parities
    base = quant.bf16(r.standard_normal(2000).astype(np.float32))
    ulp = np.abs(base).view(np.uint32)
    tie = ((ulp + 0x8000).view(np.float32) * np.sign(base)).astype(np.float32)
    x = np.concatenate([x, tie, np.float32([0.0, -0.0, 1.0, 65504.0])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(quant.bf16(x), ref)


def test_quantiser_properties():
    m = np.float32(3.7)
    x = np.float32([0.0, 3.7, -3.7, 1e-9, -1e-9])
    q = quant.quantise(x, m)
    np.testing.assert_array_equal(q, [0, 127, -127, 0, 0])
    k = np.arange(-127, 128, dtype=np.float32)
    np.testing.assert_array_equal(quant.quantise(k * (m / np.float32(127)), m), k)
    r = np.random.default_rng(1)
    y = r.uniform(-3.7, 3.7, 1000).astype(np.float32)
    qy = quant.quantise(y, m)
    assert np.all(np.abs(qy) <= 127) and np.array_equal(quant.quantise(-y, m), -qy)
    assert np.max(np.abs(qy * (m / 127) - y)) <= 0.5 * m / 127 * (1 + 1e-5)
    np.testing.assert_array_equal(quant.quantise(y, np.float32(0)), np.zeros_like(y))


def test_weight_quantiser_per_output_channel():
    r = np.random.default_rng(2)
    w = r.standard_normal((5, 3, 3, 3)).astype(np.float32)
    w[2] = 0.0
    q, s = quant.quantise_weights(w)
    for o in (0, 1, 3, 4):
        assert np.max(np.abs(q[o])) == 127
        assert s[o] == np.float32(np.max(np.abs(w[o]))) / np.float32(127)
    assert np.all(q[2] == 0) and s[2] == 0
    np.testing.assert_allclose(q * s[:, None, None, None], w, atol=float(np.max(s)) * 0.5 + 1e-7)


@pytest.mark.parametrize("stride,k", [(1, 3), (2, 3), (1, 1)])
def test_integer_conv_matches_fp64_conv_of_dequantised_codes(stride, k):
    r = np.random.default_rng(3 + stride + k)
    x = r.uniform(-2, 2, (2, 6, 9, 11)).astype(np.float32)
    w = r.standard_normal((7, 6, k, k)).astype(np.float32)
    b = r.standard_normal(7).astype(np.float32)
    m = np.float32(np.max(np.abs(x)))
    y, _, acc = quant.qconv(x, m, w, b, stride, act=False, store_bf16=False)
    xq = quant.quantise(x, m).astype(np.float64) * float(quant.input_scale(m))
    wq, sw = quant.quantise_weights(w)
    ref = oracle.conv2d(xq, wq.astype(np.float64) * sw[:, None, None, None].astype(np.float64),
                        b.astype(np.float64), stride, (k - 1) // 2)
    assert np.all(np.abs(acc) <= 127 * 127 * 6 * k * k)
    np.testing.assert_allclose(y, ref, rtol=4e-7, atol=4e-7 * np.max(np.abs(ref)))


@pytest.mark.parametrize("Hi,Wi,Ho,Wo", [(4, 5, 8, 9), (12, 39, 24, 78), (3, 3, 3, 3), (1, 2, 5, 7)])
def test_fp32_resize_matches_fp64(Hi, Wi, Ho, Wo):
    x = np.random.default_rng(Hi * Wo).standard_normal((2, 3, Hi, Wi)).astype(np.float32)
    np.testing.assert_allclose(quant.resize_f32(x, Ho, Wo), oracle.resize(x.astype(np.float64), Ho, Wo),
                               rtol=0, atol=4e-7 * np.max(np.abs(x)))


def _levels(H, W, f):
    h, w = [-(-H // f)], [-(-W // f)]
    for _ in range(3):
        h.append(-(-h[-1] // 2))
        w.append(-(-w[-1] // 2))
    return h, w


def _decoder_resizes():
    """(n_in, n_out) of every decoder resize axis of the 1242x375 (f = 4) and
    256x128 (f = 2) workloads and of the widest / narrowest uneven pairs."""
    out = set()
    for H, W, f in ((375, 1242, 4), (128, 256, 2), (384, 1280, 4), (192, 640, 4), (376, 1048, 4)):
        h, w = _levels(H, W, f)
        for k in range(3):
            out.add((h[k + 1], h[k]))
            out.add((w[k + 1], w[k]))
    return sorted(out)


def _rn_even_f32(q):
    """Round a rational 0 <= q < 2 to binary32, nearest with ties to even, by
    integer arithmetic: scale to a 24-bit significand and let Fraction's
    round() (half to even) pick the integer."""
    if q == 0:
        return np.float32(0)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    if Fraction(2) ** e > q:
        e -= 1
    assert Fraction(2) ** e <= q < Fraction(2) ** (e + 1)
    m = round(q * Fraction(2) ** (23 - e))
    return np.float32(float(m * Fraction(2) ** (e - 23)))


def _axis_reference(o, n_in, n_out):
    """Half-pixel source position o -> ((2o+1) n_in - n_out) / (2 n_out),
    clamped at 0: integer floor, clamped upper corner, rounded remainder."""
    num, den = (2 * o + 1) * n_in - n_out, 2 * n_out
    if num < 0:
        num = 0
    i0 = num // den
    return i0, min(i0 + 1, n_in - 1), _rn_even_f32(Fraction(num - i0 * den, den))


@pytest.mark.parametrize("n_in,n_out", _decoder_resizes() + [(3, 7), (5, 2), (1, 4), (7, 7)])
def test_bilinear_weights_are_the_correctly_rounded_exact_fraction(n_in, n_out):
    for o in range(n_out):
        got = quant._bilin_axis(o, n_in, n_out)
        ref = _axis_reference(o, n_in, n_out)
        assert got[:2] == ref[:2], (o, got, ref)
        assert np.float32(got[2]).view(np.uint32) == ref[2].view(np.uint32), (o, got[2], ref[2])


def test_fp32_expression_weights_would_fail_the_pin():
    """The pin discriminates: evaluating the position as the FP32 expression
    (o + 1/2) n_in / n_out - 1/2 rounds differently on a large share of the
    workload's indices, and every such index differs from the reference."""
    F = np.float32
    differ = total = 0
    for n_in, n_out in _decoder_resizes():
        for o in range(n_out):
            s = max((F(o) + F(0.5)) * F(n_in) / F(n_out) - F(0.5), F(0))
            lam = F(s - np.floor(s))
            total += 1
            differ += int(lam.view(np.uint32) != _axis_reference(o, n_in, n_out)[2].view(np.uint32))
    assert differ > total // 10, (differ, total)


@pytest.mark.parametrize("Hi,Wi,Ho,Wo", [(12, 39, 24, 78), (24, 78, 47, 156), (47, 156, 94, 311),
                                         (16, 32, 32, 64), (3, 5, 7, 2)])
def test_fp32_resize_bitwise_equals_scalar_definition(Hi, Wi, Ho, Wo):
    """Every output of resize_f32 equals a scalar FP32 evaluation of
    (1-ly)((1-lx) x00 + lx x01) + ly((1-lx) x10 + lx x11), each operation
    rounded, with the reference weights and corners."""
    F = np.float32
    x = np.random.default_rng(Hi * 1000 + Wo).standard_normal((1, 2, Hi, Wi)).astype(np.float32)
    got = quant.resize_f32(x, Ho, Wo)
    ys = [_axis_reference(o, Hi, Ho) for o in range(Ho)]
    xs = [_axis_reference(o, Wi, Wo) for o in range(Wo)]
    ref = np.empty((1, 2, Ho, Wo), np.float32)
    one = F(1)
    for c in range(2):
        xc = x[0, c]
        for oy, (y0, y1, ly) in enumerate(ys):
            wy0 = F(one - ly)
            for ox, (x0, x1, lx) in enumerate(xs):
                wx0 = F(one - lx)
                top = F(F(wx0 * xc[y0, x0]) + F(lx * xc[y0, x1]))
                bot = F(F(wx0 * xc[y1, x0]) + F(lx * xc[y1, x1]))
                ref[0, c, oy, ox] = F(F(wy0 * top) + F(ly * bot))
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))


def _shapes(C, L):
    return [(o, i, k) for (o, i, k, s) in vae.layer_shapes(*C, L)]


def test_bias_only_network_reduces_to_the_fp_network():
    # zero weights: every integer sum is 0, each layer stores lrelu(bias); with
    # non-negative BF16-representable biases the INT8 pass is the FP network exactly
    C, L, f, H, W = (8, 16, 16), 8, 2, 24, 40
    r = np.random.default_rng(4)
    params = []
    for (o, i, k) in _shapes(C, L):
        b = quant.bf16(r.uniform(0, 1, o).astype(np.float32))
        params.append((np.zeros((o, i, k, k), np.float32), b))
    wF = r.standard_normal((1, C[0] + 2, 3, 3)).astype(np.float32)
    params[8] = (wF, params[8][1])
    d = r.integers(0, 30, (2, 12, 20)).astype(np.uint8)
    im = r.integers(0, 256, (2, 12, 20)).astype(np.uint8)
    tq = quant.forward(params, d, im, f, H, W)
    t64 = vae.forward(params, d, im, f, H, W)
    np.testing.assert_allclose(tq["out"], t64["out"], rtol=0, atol=1e-9)
    np.testing.assert_array_equal(tq["mu"], t64["mu"].astype(np.float32))


def test_int8_network_is_close_to_fp64():
    C, L, f, H, W = (16, 32, 64), 64, 2, 64, 128
    params = he_init_params(_shapes(C, L), seed=7001, bias_scale=0.1)
    r = np.random.default_rng(5)
    d = r.integers(0, 16, (1, 32, 64)).astype(np.uint8)
    im = r.integers(0, 256, (1, 32, 64)).astype(np.uint8)
    tq = quant.forward(params, d, im, f, H, W)
    t64 = vae.forward(params, d, im, f, H, W)
    R = t64["out"] - 256.0 * t64["base"]
    err = np.mean(np.abs(tq["out"] - t64["out"]))
    # quantisation noise of a few per cent of the refinement term, nowhere near its size
    assert err <= 0.1 * np.mean(np.abs(R)), (err, np.mean(np.abs(R)))
    for k in ("E1", "E2", "E3", "G3", "G2", "G1", "G0"):
        assert np.array_equal(quant.bf16(tq[k]), tq[k])
