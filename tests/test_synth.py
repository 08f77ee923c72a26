"""Seeded generator: determinism, ranges and warp consistency."""
import numpy as np

from synth import gen_pair, gen_preset, gen_shift_pair, he_init_params, gen_eps


def test_deterministic_per_seed():
    a, b = gen_pair(64, 96, 4, 2.0, 20.0, seed=5), gen_pair(64, 96, 4, 2.0, 20.0, seed=5)
    assert (a.left == b.left).all() and (a.right == b.right).all() and (a.gt == b.gt).all()
    c = gen_pair(64, 96, 4, 2.0, 20.0, seed=6)
    assert not (a.left == c.left).all()


def test_ranges_and_masks():
    p = gen_preset("pair256x128")
    assert p.left.shape == (128, 256) and p.left.dtype == np.uint8
    assert p.gt.min() >= 4.0 - 1e-5 and p.gt.max() <= 24.0 + 1e-5
    assert p.occ.all() and 0.5 < p.noc.mean() < 1.0
    p2 = gen_preset("pair1242x375")
    assert p2.left.shape == (375, 1242) and p2.D == 48 and p2.gt.max() <= 190.0 + 1e-4


def test_warp_consistency_on_visible_pixels():
    """A visible left pixel lands on x' = floor(x - d + 1/2) in the right view, up
    to the sensor noise (sigma 2, so 6 sigma = 12 grey levels)."""
    p = gen_pair(96, 160, 5, 3.0, 30.0, seed=9)
    ys, xs = np.nonzero(p.noc)
    xt = np.floor(xs - p.gt[ys, xs] + 0.5).astype(int)
    diff = np.abs(p.right[ys, xt].astype(int) - p.left[ys, xs].astype(int))
    assert np.percentile(diff, 99.9) <= 12


def test_uneven_batch_sizes():
    sizes = [gen_preset("uneven64", i).left.shape for i in range(4)]
    for (H, W) in sizes:
        assert H % 8 == 0 and W % 8 == 0 and 192 <= H <= 384 and 640 <= W <= 1280
    assert len(set(sizes)) > 1


def test_shift_pair():
    p = gen_shift_pair(32, 64, 6, seed=1)
    assert (p.right[:, :58] == p.left[:, 6:]).all()


def test_weights_and_eps():
    ps = he_init_params([(4, 2, 3), (1, 4, 1)], seed=3)
    assert ps[0][0].shape == (4, 2, 3, 3) and ps[1][0].shape == (1, 4, 1, 1)
    assert (ps[0][1] == 0).all()
    assert abs(np.std(he_init_params([(64, 64, 3)], seed=4)[0][0]) - np.sqrt(2 / 576)) < 0.005
    e = gen_eps((1, 5, 3, 3), seed=9000)
    assert e.dtype == np.float32 and (e == gen_eps((1, 5, 3, 3), seed=9000)).all()
