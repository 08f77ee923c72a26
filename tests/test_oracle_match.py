"""Pins of the oracle's matching stage (downsample, census, Hamming cost, WTA).

Each check rests on something other than the oracle itself: closed forms,
invariants, a hand-worked fixture, numpy reductions, or brute force written as
a different computation on tiny inputs.
"""
import os

import numpy as np
import pytest

import oracle
from synth import gen_pair, gen_shift_pair, gen_preset

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _offsets(ww, wh):
    rx, ry = (ww - 1) // 2, (wh - 1) // 2
    return [(dy, dx) for dy in range(-ry, ry + 1) for dx in range(-rx, rx + 1) if (dy, dx) != (0, 0)]


# ---------------------------------------------------------------- downsample

@pytest.mark.parametrize("f", [1, 2, 3, 4])
def test_downsample_constant_and_identity(f):
    img = np.full((1, 13, 9), 77, np.uint8)
    assert (oracle.downsample(img, f) == 77).all()
    rng = np.random.default_rng(f)
    img = rng.integers(0, 256, (2, 13, 9), dtype=np.uint8)
    if f == 1:
        assert (oracle.downsample(img, 1) == img).all()


@pytest.mark.parametrize("f", [2, 3, 4])
def test_downsample_block_mean_numpy(f):
    """Full blocks: numpy reshape-mean with round-half-up; partial edge blocks: mean
    of their in-bounds pixels (padded with NaN and nanmean)."""
    rng = np.random.default_rng(10 + f)
    img = rng.integers(0, 256, (2, 13, 9), dtype=np.uint8)
    h, w = -(-13 // f), -(-9 // f)
    pad = np.full((2, h * f, w * f), np.nan)
    pad[:, :13, :9] = img
    blocks = pad.reshape(2, h, f, w, f)
    s = np.nansum(blocks, axis=(2, 4))
    n = np.sum(~np.isnan(blocks), axis=(2, 4))
    expect = np.floor((s + np.floor(n / 2)) / n).astype(np.uint8)
    assert (oracle.downsample(img, f) == expect).all()


def test_downsample_round_half_up():
    img = np.array([[[1, 2], [2, 2]]], np.uint8)   # sum 7, n 4 -> 7/4 = 1.75 -> 2
    assert oracle.downsample(img, 2)[0, 0, 0] == 2
    img = np.array([[[1, 2], [1, 2]]], np.uint8)   # 6/4 = 1.5 -> 2 (half up)
    assert oracle.downsample(img, 2)[0, 0, 0] == 2
    img = np.array([[[1, 1], [1, 2]]], np.uint8)   # 5/4 = 1.25 -> 1
    assert oracle.downsample(img, 2)[0, 0, 0] == 1


# ------------------------------------------------------------------- census

def test_census_hand_worked_fixture():
    img = np.array([[10, 20, 30, 40, 50],
                    [60, 70, 80, 90, 100],
                    [15, 25, 35, 45, 55],
                    [65, 75, 85, 95, 105],
                    [10, 10, 10, 10, 10]], np.uint8)
    c = oracle.census(img, 3, 3)[0]
    rows = [l.split() for l in open(os.path.join(GOLDEN, "census_5x5_win3.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for r, col, val in rows:
        assert int(c[int(r), int(col)]) == int(val)


@pytest.mark.parametrize("ww,wh", [(5, 5), (9, 7), (3, 3)])
def test_census_constant_zero(ww, wh):
    assert (oracle.census(np.full((9, 11), 100, np.uint8), ww, wh) == 0).all()


@pytest.mark.parametrize("ww,wh", [(5, 5), (9, 7)])
def test_census_ramps_closed_form(ww, wh):
    """Horizontal strict ramp I = x: bit k = [dx_k < 0] where the window is interior;
    vertical ramp I = y: bit k = [dy_k < 0]."""
    h, w = 15, 20
    offs = _offsets(ww, wh)
    rx, ry = (ww - 1) // 2, (wh - 1) // 2
    horiz = np.tile(np.arange(w, dtype=np.uint8) * 3, (h, 1))
    vert = np.tile((np.arange(h, dtype=np.uint8) * 5)[:, None], (1, w))
    eh = sum(1 << k for k, (dy, dx) in enumerate(offs) if dx < 0)
    ev = sum(1 << k for k, (dy, dx) in enumerate(offs) if dy < 0)
    ch = oracle.census(horiz, ww, wh)[0]
    cv = oracle.census(vert, ww, wh)[0]
    assert (ch[:, rx:w - rx] == eh).all()
    assert (cv[ry:h - ry, :] == ev).all()
    # at the left border the clamped neighbours equal the centre: those bits are 0
    eh0 = sum(1 << k for k, (dy, dx) in enumerate(offs) if dx < 0 and False)
    assert (ch[:, 0] == eh0).all()


def test_census_popcount_counts_darker_neighbours():
    """popcount(code) = number of window cells strictly darker than the centre
    (computed with a padded-array comparison, not bit by bit)."""
    rng = np.random.default_rng(3)
    img = rng.integers(0, 6, (12, 17), dtype=np.uint8)   # many equal values
    ww, wh = 9, 7
    c = oracle.census(img, ww, wh)[0]
    rx, ry = 4, 3
    pad = np.pad(img.astype(int), ((ry, ry), (rx, rx)), mode="edge")
    cnt = np.zeros_like(img, dtype=int)
    for dy in range(-ry, ry + 1):
        for dx in range(-rx, rx + 1):
            cnt += pad[ry + dy:ry + dy + 12, rx + dx:rx + dx + 17] < img
    pc = np.array([bin(int(v)).count("1") for v in c.ravel()]).reshape(c.shape)
    assert (pc == cnt).all()
    assert int(c.max()) < (1 << (ww * wh - 1))


def test_census_brute_force_tiny():
    rng = np.random.default_rng(4)
    img = rng.integers(0, 256, (2, 6, 7), dtype=np.uint8)
    ww, wh = 5, 3
    c = oracle.census(img, ww, wh)
    for b in range(2):
        for i in range(6):
            for j in range(7):
                bits = ""
                for dy, dx in _offsets(ww, wh):
                    y, x = min(max(i + dy, 0), 5), min(max(j + dx, 0), 6)
                    bits = ("1" if img[b, y, x] < img[b, i, j] else "0") + bits
                assert int(c[b, i, j]) == int(bits, 2)


# -------------------------------------------------------------- Hamming cost

def test_hamming_identities():
    rng = np.random.default_rng(5)
    nbits = 62
    mask = (1 << nbits) - 1
    a = rng.integers(0, 1 << 62, (1, 4, 9), dtype=np.uint64)
    b = rng.integers(0, 1 << 62, (1, 4, 9), dtype=np.uint64)
    caa = oracle.cost_volume(a, a, 1, nbits)[..., 0]
    assert (caa == 0).all()
    cab = oracle.cost_volume(a, b, 1, nbits)[..., 0]
    cba = oracle.cost_volume(b, a, 1, nbits)[..., 0]
    assert (cab == cba).all()
    na = (~a) & np.uint64(mask)
    assert (oracle.cost_volume(a, na, 1, nbits)[..., 0] == nbits).all()


def test_cost_volume_brute_force_and_sentinel():
    rng = np.random.default_rng(6)
    cl = rng.integers(0, 1 << 24, (1, 8, 16), dtype=np.uint64)
    cr = rng.integers(0, 1 << 24, (1, 8, 16), dtype=np.uint64)
    D, nbits = 7, 24
    cv = oracle.cost_volume(cl, cr, D, nbits)
    for i in range(8):
        for j in range(16):
            for d in range(D):
                if j - d < 0:
                    assert cv[0, i, j, d] == nbits + 1
                else:
                    x = int(cl[0, i, j]) ^ int(cr[0, i, j - d])
                    assert cv[0, i, j, d] == bin(x).count("1")


# ---------------------------------------------------------------------- WTA

def test_wta_lowest_index_on_ties():
    cost = np.array([[[[5, 3, 3, 4], [2, 2, 2, 2], [9, 8, 7, 1]]]], np.int32)
    assert oracle.wta(cost).tolist() == [[[1, 0, 3]]]
    rng = np.random.default_rng(7)
    cost = rng.integers(0, 4, (1, 5, 6, 9)).astype(np.int32)
    ref = np.array([[[min(range(9), key=lambda d: (cost[0, i, j, d], d)) for j in range(6)]
                     for i in range(5)]])
    assert (oracle.wta(cost) == ref).all()


def test_identical_images_give_zero_disparity():
    p = gen_pair(64, 96, 4, 2.0, 10.0, seed=11)
    _, _, _, d = oracle.match(p.left, p.left, 2, 5, 5, 16)
    assert (d == 0).all()


@pytest.mark.parametrize("shift,f,ww,wh,D", [(8, 2, 5, 5, 16), (12, 4, 9, 7, 8), (20, 4, 9, 7, 12)])
def test_integer_shift_recovered(shift, f, ww, wh, D):
    """right(x) = left(x + s) with s a multiple of f: d = s/f wherever both census
    windows are interior and filled from the shifted texture; any exception must
    be a genuine lower-disparity tie (checked on the full cost volume)."""
    H, W = 96, 192
    p = gen_shift_pair(H, W, shift, seed=21 + shift)
    lo_l, cl, cr, d = oracle.match(p.left, p.right, f, ww, wh, D)
    s = shift // f
    nbits = ww * wh - 1
    cv = oracle.cost_volume(cl, cr, D, nbits)[0]
    h, w = lo_l.shape[1:]
    rx, ry = (ww - 1) // 2, (wh - 1) // 2
    valid_right_cols = (W - shift) // f          # low-res right columns fully from left texture
    checked = 0
    for i in range(ry, h - ry):
        for j in range(s + rx, min(w - rx, valid_right_cols - rx + s)):
            assert cv[i, j, s] == 0
            if d[0, i, j] != s:
                assert d[0, i, j] < s and cv[i, j, d[0, i, j]] == 0
            checked += 1
    assert checked > 100
    frac = np.mean(d[0, ry:h - ry, s + rx:w - rx] == s)
    assert frac > 0.9


def test_disparity_never_exceeds_column():
    p = gen_preset("pair256x128")
    _, _, _, d = oracle.match(p.left, p.right, 2, 5, 5, 16)
    j = np.arange(d.shape[2])[None, None, :]
    assert (d <= j).all()
