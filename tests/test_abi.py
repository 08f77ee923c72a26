"""C ABI: the library loads, exports every symbol the header declares, and
rejects bad arguments before touching the GPU (runs without a GPU)."""
import ctypes

import pytest

import paper_2305_11566_amd as sv
from paper_2305_11566_amd._lib import lib, header_symbols, make_desc


def test_exports_every_declared_symbol():
    l = lib()
    missing = [s for s in header_symbols() if not hasattr(l, s)]
    assert not missing, missing


def test_status_strings():
    assert lib().sv_status_str(0) == b"SV_OK"
    assert lib().sv_status_str(-5) == b"SV_ERR_WORKSPACE"


def test_param_counts_match_workload_shapes():
    assert sv.vae_param_count(16, 32, 64, 64) == 73299
    assert sv.vae_param_count(32, 64, 128, 128) == 290963


P = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


@pytest.mark.parametrize("args,code", [
    ((None, 1, 8, 8, 8, 2, 5, 5, None, P, None), -1),
    ((P, 0, 8, 8, 8, 2, 5, 5, None, P, None), -2),
    ((P, 1, 8, 8, 4, 2, 5, 5, None, P, None), -2),       # pitch < W
    ((P, 1, 8, 8, 8, 9, 5, 5, None, P, None), -3),       # factor
    ((P, 1, 8, 8, 8, 2, 4, 5, None, P, None), -3),       # even window
    ((P, 1, 8, 8, 8, 2, 9, 9, None, P, None), -3),       # nbits 80 > 64
    ((P, 1, 8, 8, 8, 2, 19, 3, None, P, None), -3),      # window wider than 17
])
def test_census_validation(args, code):
    assert lib().sv_census(*args) == code


@pytest.mark.parametrize("args,code", [
    ((None, P, 1, 4, 4, 8, 24, P, None), -1),
    ((P, P, 1, 0, 4, 8, 24, P, None), -2),
    ((P, P, 1, 4, 4, 257, 24, P, None), -3),
    ((P, P, 1, 4, 4, 0, 24, P, None), -3),
    ((P, P, 1, 4, 4, 8, 65, P, None), -3),
])
def test_cost_wta_validation(args, code):
    assert lib().sv_cost_wta(*args) == code


@pytest.mark.parametrize("args,code", [
    ((None, P, 1, 4, 4, 8, 24, 10, 120, P, P, 1024, None), -1),
    ((P, P, 1, 4, 4, 8, 24, 10, 120, P, None, 1024, None), -1),
    ((P, P, 1, 0, 4, 8, 24, 10, 120, P, P, 1024, None), -2),
    ((P, P, 1, 4, 4, 257, 24, 10, 120, P, P, 10 ** 6, None), -3),
    ((P, P, 1, 4, 4, 8, 24, 10, 5, P, P, 1024, None), -3),      # P2 < P1
    ((P, P, 1, 4, 4, 8, 24, -1, 120, P, P, 1024, None), -3),    # P1 < 0
    ((P, P, 1, 4, 4, 8, 62, 10, 193, P, P, 1024, None), -3),    # path costs beyond uint8
    ((P, P, 1, 4, 4, 8, 24, 10, 120, P, P, 4 * 4 * 4 * 8 - 1, None), -5),
])
def test_sgm_validation(args, code):
    assert lib().sv_sgm(*args) == code


@pytest.mark.parametrize("args,code", [
    ((None, 1, 4, 4, 8, P, P, 16, None), -1),
    ((P, 1, 4, 4, 8, P, None, 16, None), -1),
    ((P, 1, 4, 16385, 8, P, P, 10 ** 6, None), -2),
    ((P, 1, 4, 4, 0, P, P, 16, None), -3),
    ((P, 1, 4, 4, 8, P, P, 15, None), -5),
])
def test_smp_median_validation(args, code):
    assert lib().sv_smp_median(*args) == code


@pytest.mark.parametrize("args,code", [
    ((None, P, 1, 4, 4, 8, 5, 5, 10, 120, P, P, 10 ** 6, None), -1),
    ((P, P, 1, 0, 4, 8, 5, 5, 10, 120, P, P, 10 ** 6, None), -2),
    ((P, P, 1, 4, 4, 8, 4, 5, 10, 120, P, P, 10 ** 6, None), -3),     # even window
    ((P, P, 1, 4, 4, 8, 5, 5, 10, 192, P, P, 10 ** 6, None), -3),     # 64 + P2 > 255
    ((P, P, 1, 4, 4, 8, 5, 5, 10, 120, P, P, 10, None), -5),
])
def test_zncc_sgm_validation(args, code):
    assert lib().sv_zncc_sgm(*args) == code


def test_vae_validation():
    l = lib()
    d = make_desc(16, 32, 64, 64, 2, "f32")
    ws = l.sv_vae_workspace_bytes(ctypes.byref(d), 1, 128, 256)
    assert ws > 0
    A = ctypes.c_void_p(0x100000)
    # workspace too small
    assert l.sv_vae_forward(ctypes.byref(d), A, P, P, 1, 128, 256, None, P, None, None, A, ws - 1, None) == -5
    # training without a saved buffer
    assert l.sv_vae_forward(ctypes.byref(d), A, P, P, 1, 128, 256, P, P, None, None, A, ws, None) == -1
    # misaligned workspace
    assert l.sv_vae_forward(ctypes.byref(d), A, P, P, 1, 128, 256, None, P, None, None,
                            ctypes.c_void_p(0x100010), ws, None) == -3
    bad = make_desc(12, 32, 64, 64, 2, "f32")      # not a multiple of 8
    assert l.sv_vae_param_count(ctypes.byref(bad)) == -3
    bad = make_desc(16, 32, 64, 64, 2, 7)
    assert l.sv_vae_param_count(ctypes.byref(bad)) == -4
    assert l.sv_vae_workspace_bytes(ctypes.byref(d), 0, 128, 256) == 0


def test_int8_is_inference_only():
    l = lib()
    d = make_desc(16, 32, 64, 64, 2, "i8")
    d16 = make_desc(16, 32, 64, 64, 2, "bf16")
    assert l.sv_vae_param_count(ctypes.byref(d)) == 73299
    assert 0 < l.sv_vae_packed_bytes(ctypes.byref(d)) < l.sv_vae_packed_bytes(ctypes.byref(d16))
    ws = l.sv_vae_workspace_bytes(ctypes.byref(d), 1, 128, 256)
    assert ws > 0
    A = ctypes.c_void_p(0x100000)
    # eps / saved (training) -> unsupported; backward -> unsupported
    assert l.sv_vae_forward(ctypes.byref(d), A, P, P, 1, 128, 256, P, P, None, A, A, ws, None) == -6
    assert l.sv_vae_forward(ctypes.byref(d), A, P, P, 1, 128, 256, None, P, None, A, A, ws, None) == -6
    assert l.sv_vae_backward(ctypes.byref(d), A, A, 1, 128, 256, None, P, None, ctypes.c_float(0.0),
                             P, A, ws, None) == -6
    plan = ctypes.c_void_p()
    assert l.sv_batch_plan_create(ctypes.byref(d), 4, 128, 256, 16, 5, 5, ctypes.byref(plan)) == -6


def test_tvae_counts_and_sizes():
    from oracle import tvae
    assert lib().sv_tvae_param_count() == tvae.n_params() == 162380
    assert lib().sv_tvae_packed_bytes(0) > 0 and lib().sv_tvae_packed_bytes(7) == 0
    assert lib().sv_tvae_packed_bytes(0) % 256 == 0
    assert lib().sv_tvae_workspace_bytes(0, 4, 1, 375, 1242) > 0
    assert lib().sv_tvae_workspace_bytes(0, 9, 1, 375, 1242) == 0    # factor
    assert lib().sv_tvae_workspace_bytes(0, 4, 0, 375, 1242) == 0    # batch
    assert lib().sv_tvae_workspace_bytes(5, 4, 1, 375, 1242) == 0    # dtype
    assert lib().sv_tvae_workspace_bytes(0, 4, 16384, 64, 64) == 0   # grid z limit
    assert lib().sv_tvae_num_layers() == 12


@pytest.mark.parametrize("args,code", [
    ((0, 4, None, P, P, 1, 64, 64, None, P, None, P, 1 << 30, None), -1),
    ((0, 4, P, P, P, 1, 64, 64, None, None, None, P, 1 << 30, None), -1),
    ((7, 4, P, P, P, 1, 64, 64, None, P, None, P, 1 << 30, None), -4),
    ((0, 0, P, P, P, 1, 64, 64, None, P, None, P, 1 << 30, None), -3),
    ((0, 4, P, P, P, 0, 64, 64, None, P, None, P, 1 << 30, None), -2),
    ((0, 4, P, P, P, 1, 64, 64, None, P, None, P, 16, None), -5),
])
def test_tvae_forward_validation(args, code):
    assert lib().sv_tvae_forward(*args) == code


def test_tvae_loss_and_cfg_validation():
    nb = lib().sv_tvae_loss_workspace_bytes()
    assert lib().sv_tvae_loss(None, P, P, P, 10, P, 2, P, None, None, P, nb, None) == -1
    assert lib().sv_tvae_loss(P, P, P, P, 0, P, 2, P, None, None, P, nb, None) == -2
    assert lib().sv_tvae_loss(P, P, P, P, 10, P, 2, P, None, None, P, 8, None) == -5
    assert lib().sv_tvae_set_layer_cfg(12, 0) == -3
    assert lib().sv_tvae_set_layer_cfg(0, lib().sv_num_layer_cfgs()) == -3
    assert lib().sv_tvae_set_layer_cfg(0, -1) == 0
    assert lib().sv_tvae_autotune(7, 4, 1, 64, 64) == -4
    assert lib().sv_tvae_autotune(0, 9, 1, 64, 64) == -3
    assert lib().sv_tvae_layer_cfgs(0, 4, 1, 64, 64, None) == -1
    arr = (ctypes.c_int * 12)()
    assert lib().sv_tvae_layer_cfgs(0, 4, 1, 375, 1242, arr) == 0
    assert all(0 <= c < lib().sv_num_layer_cfgs() for c in arr)


def test_latent_fusion_switch():
    assert lib().sv_set_latent_fusion(2) == -3
    assert lib().sv_set_latent_fusion(-1) == -3
    assert lib().sv_set_latent_fusion(0) == 0
    assert lib().sv_set_latent_fusion(1) == 0


def test_paper_batch_validation():
    """sv_paper_batch checks its settings and every pair before any launch
    (dummy device pointers: nothing is dereferenced)."""
    from paper_2305_11566_amd._lib import PaperDesc, Pair
    ok = PaperDesc(0, 2, 5, 5, 10, 120, 1, 0)
    need = lib().sv_paper_batch_workspace_bytes(ctypes.byref(ok), 128, 256, 16)
    assert need > 0
    assert lib().sv_paper_batch_workspace_bytes(ctypes.byref(PaperDesc(2, 2, 5, 5, 10, 120, 1, 0)), 128, 256, 16) == 0
    dummy, ws = 0x10000, 0x20000
    pairs = (Pair * 1)(Pair(dummy, dummy, dummy, None, 128, 256, 16))
    call = lambda d, pr=pairs, n=1, w=ws, nb=need: lib().sv_paper_batch(ctypes.byref(d), pr, n, dummy, w, nb, None)
    assert call(PaperDesc(2, 2, 5, 5, 10, 120, 1, 0)) == -3           # matcher
    assert call(PaperDesc(0, 9, 5, 5, 10, 120, 1, 0)) == -3           # factor
    assert call(PaperDesc(0, 2, 5, 5, 10, 200, 1, 0)) == -3           # ZNCC: 64 + P2 > 255
    assert call(PaperDesc(1, 2, 5, 5, 10, 240, 1, 0)) == -3           # census: nbits + 1 + P2 > 255
    assert call(PaperDesc(0, 2, 5, 5, 20, 10, 1, 0)) == -3            # P2 < P1
    assert call(PaperDesc(0, 2, 7, 5, 10, 120, 1, 0)) == -6           # no ZNCC kernel for 7x5
    assert call(PaperDesc(0, 2, 5, 5, 10, 120, 1, 3)) == -4           # INT8 network not offered
    assert lib().sv_paper_batch(ctypes.byref(ok), None, 1, dummy, ws, need, None) == -1
    assert call(ok, pr=(Pair * 1)(Pair(dummy, dummy, dummy, None, 0, 256, 16))) == -2
    assert call(ok, pr=(Pair * 1)(Pair(dummy, dummy, dummy, None, 128, 256, 300))) == -2
    assert call(ok, pr=(Pair * 1)(Pair(dummy, dummy, dummy, None, 256, 512, 16))) == -5   # larger than sized for
    assert call(ok, w=ws + 16) == -3                                   # misaligned workspace


def test_profile_repeat_range():
    assert lib().sv_profile_repeat(0) == -3
    assert lib().sv_profile_repeat(65) == -3
    assert lib().sv_profile_repeat(64) == 0
    assert lib().sv_profile_repeat(1) == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_2305_11566_amd._lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="not built"):
        L.lib()
