"""GPU parity of the Table I network (Sec. III-B1) and its loss (Eqs. (9)-(11))
against the FP64 oracle.

FP32: normwise max|y - y64| / max|y64| <= 1e-5 on the refined disparity and on
mu / sigma.  BF16 / FP16: mean end-point error bounded relative to the output
scale.  Tile shapes must not change a single bit.  The loss: value within
1e-6 relative, gradients within 1e-6 normwise.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import tvae
from synth import gen_preset, gen_pair, gen_eps, he_init_params
from tests.gpu_util import cuda, flat_params, normwise

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


def _params(seed, bias_scale=0.1):
    return he_init_params(tvae.layer_shapes(), seed=seed, bias_scale=bias_scale)


def _latent_hw(H, W, f):
    h, w = -(-H // f), -(-W // f)
    for _ in range(2):
        h, w = -(-h // 2), -(-w // 2)
    return h, w


def _gpu(dtype, f, params, disp, img, H, W, eps=None):
    import paper_2305_11566_amd as sv
    net = sv.TableVAE(f, dtype)
    net.pack(cuda(flat_params(params)))
    out, ms = net.forward(cuda(disp), cuda(img), H, W, eps=None if eps is None else cuda(eps))
    torch.cuda.synchronize()
    return out.cpu().numpy(), ms.cpu().numpy()


def _compare(f, H, W, disp, img, seed=7, eps=None, dtype="f32", tol=TOL_F32):
    params = _params(seed)
    t = tvae.forward(params, disp, img, f, H, W, eps=None if eps is None else eps[:, None])
    out, ms = _gpu(dtype, f, params, disp, img, H, W, eps)
    e_out = normwise(out, t["out"])
    e_ms = max(normwise(ms[..., 0], t["mu"][:, 0]), normwise(ms[..., 1], t["sigma"][:, 0]))
    assert e_out <= tol, f"out normwise {e_out:.3e}"
    assert e_ms <= tol, f"mu/sigma normwise {e_ms:.3e}"
    return out, t


def _rand_inputs(B, H, W, f, seed):
    rng = np.random.default_rng(seed)
    h, w = -(-H // f), -(-W // f)
    return (rng.integers(0, 48, (B, h, w)).astype(np.uint8),
            rng.integers(0, 256, (B, h, w)).astype(np.uint8))


def test_f32_full_size_1242x375(deconv_form):
    p = gen_preset("pair1242x375")
    lo, _, _, d = oracle.match(p.left, p.right, 4, 9, 7, 48)
    _compare(4, 375, 1242, d, lo)


def test_f32_table_factor_2():
    p = gen_preset("pair256x128")
    lo, _, _, d = oracle.match(p.left, p.right, 2, 5, 5, 16)
    _compare(2, 128, 256, d, lo)


@pytest.fixture(params=[0, 1], ids=["zero_inserted", "polyphase"])
def deconv_form(request):
    import paper_2305_11566_amd as sv
    sv.sv_tvae_set_deconv_form(request.param)
    yield request.param
    sv.sv_tvae_set_deconv_form(-1)


@pytest.mark.parametrize("H,W,f,B", [
    (45, 70, 4, 2),     # every level ragged, odd deconvolution outputs
    (37, 53, 2, 1),
    (30, 81, 3, 2),     # stride-3 upsampling layer
    (13, 19, 1, 1),     # f = 1: the upsampling layer keeps the size
    (8, 8, 8, 3),       # coarse map 1x1: every level 1x1
    (64, 512, 4, 1),    # wide: many column tiles
    (100, 36, 2, 2),    # tall
])
def test_f32_shapes(H, W, f, B, deconv_form):
    d, im = _rand_inputs(B, H, W, f, H * W + f)
    _compare(f, H, W, d, im, seed=H)


def test_f32_training_eps(deconv_form):
    H, W, f, B = 48, 80, 2, 2
    d, im = _rand_inputs(B, H, W, f, 3)
    eps = gen_eps((B,) + _latent_hw(H, W, f), seed=9001).astype(np.float32)
    _compare(f, H, W, d, im, eps=eps)


def test_tile_shapes_bitwise_identical(deconv_form):
    # the reduction order is fixed by the base chunk and the split, not by the
    # tile shape: every tile shape gives the same bits at a given split, and a
    # split stays within the FP32 bar of the unsplit pass
    import paper_2305_11566_amd as sv
    H, W, f, B = 45, 70, 4, 2
    d, im = _rand_inputs(B, H, W, f, 17)
    params = _params(3)
    nt = sv.sv_num_layer_cfgs() // 4   # tile shapes; cfg = tile + nt * (split - 1)

    def run_all(cfg):
        for layer in range(sv.sv_tvae_num_layers()):
            sv.sv_tvae_set_layer_cfg(layer, cfg)
        return _gpu("f32", f, params, d, im, H, W)[0]

    try:
        for split in (1, 2, 4):
            base = run_all(5 + nt * (split - 1))
            if split == 1:
                unsplit = base
            else:
                assert normwise(base, unsplit) <= TOL_F32, split
            for tile in (0, 1, 3, 4, 6, 7, 9, 11, 13, 15):
                out = run_all(tile + nt * (split - 1))
                assert np.array_equal(out, base), sv.sv_conv_cfg_name(tile + nt * (split - 1))
    finally:
        for layer in range(sv.sv_tvae_num_layers()):
            sv.sv_tvae_set_layer_cfg(layer, -1)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_reduced_precision_epe(dtype, deconv_form):
    p = gen_preset("pair256x128")
    lo, _, _, d = oracle.match(p.left, p.right, 2, 5, 5, 16)
    params = _params(7)
    t = tvae.forward(params, d, lo, 2, 128, 256)
    out, _ = _gpu(dtype, 2, params, d, lo, 128, 256)
    epe = float(np.mean(np.abs(out - t["out"])))
    scale = float(np.mean(np.abs(t["out"])))
    print(f"{dtype}: mean EPE {epe:.4f} px, max {np.max(np.abs(out - t['out'])):.3f} px, mean |out| {scale:.2f}")
    # He-init weights (outputs of about 52 px): measured 0.12 px (BF16) and
    # 0.013 px (FP16); the bars leave about 1.7x of headroom
    assert epe <= {"bf16": 0.2, "f16": 0.025}[dtype]


def test_loss_matches_oracle():
    import paper_2305_11566_amd as sv
    H, W, f, B = 40, 64, 2, 2
    pairs = [gen_pair(H, W, 4, 2.0, 20.0, seed=5500 + b) for b in range(B)]
    gt = np.stack([p.gt for p in pairs]).astype(np.float32)
    noc = np.stack([p.noc for p in pairs])
    occ = np.stack([p.occ for p in pairs])
    occ[0, :3] = False          # some pixels without ground truth
    noc &= occ
    rng = np.random.default_rng(1)
    out = (gt + rng.normal(0, 2.0, gt.shape)).astype(np.float32)
    out[1, 5, 5] = gt[1, 5, 5]  # exact hit: zero gradient
    ms = rng.normal(1.0, 0.3, (B,) + _latent_hw(H, W, f) + (2,)).astype(np.float32)
    tot, l1, l2, dout, dmu, dsig = tvae.loss(out, gt, noc, occ, ms[..., 0], ms[..., 1])
    loss, gdout, gdml = sv.sv_tvae_loss(cuda(out), cuda(gt), cuda(noc.astype(np.uint8)),
                                        cuda(occ.astype(np.uint8)), cuda(ms))
    torch.cuda.synchronize()
    loss = loss.cpu().numpy().astype(np.float64)
    for got, ref in zip(loss, (tot, l1, l2)):
        assert abs(got - ref) <= 1e-6 * max(1.0, abs(ref)), (got, ref)
    assert normwise(gdout.cpu().numpy(), dout) <= 1e-6
    g = gdml.cpu().numpy()
    assert normwise(g[..., 0], dmu) <= 1e-6
    assert normwise(g[..., 1], dsig) <= 1e-6
    assert gdout.cpu().numpy()[1, 5, 5] == 0.0


def test_autotuned_pass_keeps_parity():
    import paper_2305_11566_amd as sv
    H, W, f, B = 45, 70, 4, 2
    d, im = _rand_inputs(B, H, W, f, 23)
    sv.sv_tvae_autotune("f32", f, B, H, W)
    names = sv.sv_tvae_layer_cfgs("f32", f, B, H, W)
    assert len(names) == sv.sv_tvae_num_layers() and all(n != "?" for n in names)
    _compare(f, H, W, d, im, seed=5)


def _grad_case(dtype, f, H, W, B, train, seed):
    import paper_2305_11566_amd as sv
    d, im = _rand_inputs(B, H, W, f, seed)
    params = _params(seed + 1)
    r = np.random.default_rng(seed + 2)
    h3, w3 = _latent_hw(H, W, f)
    eps = gen_eps((B, h3, w3), seed=9000 + seed).astype(np.float32) if train else None
    dout = r.standard_normal((B, H, W)).astype(np.float32)
    dms = r.standard_normal((B, h3, w3, 2)).astype(np.float32)
    t = tvae.forward(params, d, im, f, H, W, eps=None if eps is None else eps[:, None])
    ref = tvae.backward(params, t, dout, dms[..., 0][:, None], dms[..., 1][:, None])
    net = sv.TableVAE(f, dtype)
    net.pack(cuda(flat_params(params)))
    dd, ii = cuda(d), cuda(im)
    e = None if eps is None else cuda(eps)
    net.forward(dd, ii, H, W, eps=e)
    g = net.backward(dd, ii, H, W, cuda(dout), eps=e, dmu_sigma=cuda(dms))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    out, o = [], 0
    for (w_, b_) in ref:
        nw = w_.size
        out.append((g[o:o + nw].reshape(w_.shape), g[o + nw:o + nw + b_.size], w_, b_))
        o += nw + b_.size
    assert o == g.size
    return out


@pytest.mark.parametrize("f,H,W,B,train", [(2, 40, 64, 2, True), (4, 45, 70, 1, False), (3, 30, 44, 2, True)])
def test_f32_gradients_match_oracle(f, H, W, B, train):
    for name, (gw, gb, rw, rb) in zip(tvae.NAMES, _grad_case("f32", f, H, W, B, train, 40 + f)):
        ew, eb = normwise(gw, rw), normwise(gb, rb)
        assert ew <= 1e-4 and eb <= 1e-4, f"{name}: weights {ew:.2e}, bias {eb:.2e}"


def test_bf16_gradients_cosine():
    res = _grad_case("bf16", 2, 40, 64, 2, True, 60)
    allg = np.concatenate([np.concatenate([gw.ravel(), gb.ravel()]) for (gw, gb, _, _) in res])
    allr = np.concatenate([np.concatenate([rw.ravel(), rb.ravel()]) for (_, _, rw, rb) in res])
    cos = float(allg @ allr / (np.linalg.norm(allg) * np.linalg.norm(allr)))
    assert cos >= 0.999, cos
    for name, (gw, gb, rw, rb) in zip(tvae.NAMES, res):
        c = float(gw.ravel() @ rw.ravel() / max(np.linalg.norm(gw) * np.linalg.norm(rw), 1e-30))
        assert c >= 0.99, (name, c)


def test_loss_gradient_through_the_network():
    # sv_tvae_loss's gradients fed to the backward give d loss / d parameters
    import paper_2305_11566_amd as sv
    H, W, f, B = 40, 64, 2, 1
    p = gen_pair(H, W, 4, 2.0, 20.0, seed=5501)
    lo, _, _, dsp = oracle.match(p.left, p.right, f, 5, 5, 16)
    params = _params(71)
    h3, w3 = _latent_hw(H, W, f)
    eps = gen_eps((B, h3, w3), seed=9100).astype(np.float32)
    t = tvae.forward(params, dsp, lo, f, H, W, eps=eps[:, None])
    gt, noc, occ = p.gt[None].astype(np.float32), p.noc[None], p.occ[None]
    _, _, _, dout, dmu, dsig = tvae.loss(t["out"], gt, noc, occ, t["mu"][:, 0], t["sigma"][:, 0])
    ref = tvae.backward(params, t, dout, dmu[:, None], dsig[:, None])
    net = sv.TableVAE(f, "f32")
    net.pack(cuda(flat_params(params)))
    dd, ii, e = cuda(dsp), cuda(lo), cuda(eps)
    out, ms = net.forward(dd, ii, H, W, eps=e)
    loss, gdout, gdms = sv.sv_tvae_loss(out, cuda(gt), cuda(noc.astype(np.uint8)), cuda(occ.astype(np.uint8)), ms)
    g = net.backward(dd, ii, H, W, gdout, eps=e, dmu_sigma=gdms)
    torch.cuda.synchronize()
    gref = tvae.flatten([(w_, b_) for (w_, b_) in ref])
    assert normwise(g.cpu().numpy(), gref) <= 1e-3


def test_training_reduces_the_loss():
    from paper_2305_11566_amd.train import TableTrainer, make_pool, batch_indices
    params = _params(81, bias_scale=0.0)
    tr = TableTrainer(flat_params(params), factor=2, dtype="f32", lr=1e-3)
    pl, pr, pg, pn, po = make_pool(16, 64, 128, seed0=5000, masks=True)
    losses = []
    for _ in range(40):
        idx = batch_indices(tr.step, 4, 16).to(pl.device)
        losses.append(float(tr.train_step(pl[idx], pr[idx], pg[idx], pn[idx], po[idx])[0]))
    assert all(np.isfinite(losses))
    assert np.mean(losses[-5:]) < 0.8 * np.mean(losses[:5]), losses


def test_deconvolution_forms_agree():
    # the polyphase and the zero-inserted forms compute the same deconvolution
    import paper_2305_11566_amd as sv
    H, W, f, B = 45, 70, 4, 2
    d, im = _rand_inputs(B, H, W, f, 31)
    params = _params(9)
    try:
        sv.sv_tvae_set_deconv_form(0)
        a, _ = _gpu("f32", f, params, d, im, H, W)
        sv.sv_tvae_set_deconv_form(1)
        b, _ = _gpu("f32", f, params, d, im, H, W)
    finally:
        sv.sv_tvae_set_deconv_form(-1)
    assert normwise(b, a) <= 1e-6
