"""Pins of the oracle's semi-global matching (Eqs. (4)-(5)), single matching
phase (Eq. (7)) and median filter, against brute force, special cases,
symmetries and a library routine -- never against the GPU library."""
import itertools

import numpy as np
import pytest

import oracle
from synth import gen_preset


def _rand_cost(rng, B, h, w, D, hi=40):
    return rng.integers(0, hi, (B, h, w, D)).astype(np.int32)


def test_zero_penalties_reduce_to_the_matching_cost():
    # P1 = P2 = 0: every path cost equals the matching cost (Eq. (4) adds
    # min_k C_r(p - r, k) and subtracts it again), so the aggregated cost is 4 C
    # and its winner is the plain winner-take-all of Eq. (6)
    rng = np.random.default_rng(1)
    c = _rand_cost(rng, 2, 5, 7, 6)
    for r in range(4):
        assert (oracle.sgm_path(c, 0, 0, r) == c).all()
    assert (oracle.sgm(c, 0, 0) == 4 * c).all()
    assert (oracle.wta(oracle.sgm(c, 0, 0)) == oracle.wta(c)).all()


def _brute_path(costs, P1, P2):
    """Min over all disparity sequences ending in (x, d) of the summed cost and
    transition penalties (0 for the same d, P1 for a step of one, else P2;
    jumping at the cost of P2 is always allowed), for one 1-D path."""
    n, D = costs.shape
    best = np.full((n, D), np.iinfo(np.int64).max, dtype=np.int64)
    for L in range(1, n + 1):
        for seq in itertools.product(range(D), repeat=L):
            tot = sum(int(costs[i, seq[i]]) for i in range(L))
            for i in range(1, L):
                a, b = seq[i - 1], seq[i]
                pen = P2
                if a == b:
                    pen = 0
                elif abs(a - b) == 1:
                    pen = min(P1, P2)
                tot += pen
            best[L - 1, seq[-1]] = min(best[L - 1, seq[-1]], tot)
    return best


@pytest.mark.parametrize("P1,P2,seed", [(3, 9, 0), (1, 1, 1), (5, 20, 2), (0, 7, 3)])
def test_path_cost_is_the_dynamic_programme_of_its_definition(P1, P2, seed):
    # Eq. (4) is the min-sum recursion over disparity sequences along the path,
    # shifted by the running minimum: normalised per pixel, the two agree
    rng = np.random.default_rng(seed)
    n, D = 5, 3
    costs = rng.integers(0, 12, (n, D)).astype(np.int32)
    ref = _brute_path(costs, P1, P2)
    got = oracle.sgm_path(costs[None, None], P1, P2, 0)[0, 0]
    for x in range(n):
        assert (got[x] - got[x].min() == ref[x] - ref[x].min()).all(), x


def test_directions_are_mirror_images():
    rng = np.random.default_rng(4)
    c = _rand_cost(rng, 1, 6, 9, 5)
    P1, P2 = 4, 15
    l2r = oracle.sgm_path(c, P1, P2, 0)
    r2l = oracle.sgm_path(c[:, :, ::-1].copy(), P1, P2, 0)[:, :, ::-1]
    assert (oracle.sgm_path(c, P1, P2, 1) == r2l).all()
    ct = np.ascontiguousarray(c.transpose(0, 2, 1, 3))
    assert (oracle.sgm_path(c, P1, P2, 2) == oracle.sgm_path(ct, P1, P2, 0).transpose(0, 2, 1, 3)).all()
    ctf = np.ascontiguousarray(ct[:, :, ::-1])
    assert (oracle.sgm_path(c, P1, P2, 3) ==
            oracle.sgm_path(ctf, P1, P2, 0)[:, :, ::-1].transpose(0, 2, 1, 3)).all()
    assert (oracle.sgm(c, P1, P2) == l2r + oracle.sgm_path(c, P1, P2, 1) +
            oracle.sgm_path(c, P1, P2, 2) + oracle.sgm_path(c, P1, P2, 3)).all()


def test_path_costs_stay_in_the_uint8_range():
    # C_r(p, d) <= C(p, d) + P2, so with C <= nbits + 1 the GPU's uint8 volumes hold them
    rng = np.random.default_rng(5)
    c = _rand_cost(rng, 1, 8, 8, 8, hi=64)
    for r in range(4):
        pc = oracle.sgm_path(c, 10, 120, r)
        assert pc.min() >= 0 and (pc <= c + 120).all()


def test_constant_shift_recovered_on_a_textured_pair():
    # a right view that is the left one shifted by s columns: the aggregated
    # cost of d = s is 0 wherever the shifted window is inside the image
    rng = np.random.default_rng(6)
    left = rng.integers(0, 256, (1, 40, 64), dtype=np.uint8)
    s = 5
    right = np.zeros_like(left)
    right[:, :, :-s] = left[:, :, s:]
    lo_l, lo_r = oracle.downsample(left, 1), oracle.downsample(right, 1)
    cl, cr = oracle.census(lo_l, 5, 5), oracle.census(lo_r, 5, 5)
    d = oracle.wta(oracle.sgm(oracle.cost_volume(cl, cr, 12, 24), 10, 120))
    assert (d[0, 3:-3, 3 + s + 2:-3] == s).all()


def test_smp_hand_worked_row():
    # D = 4; disparities [0, 1, 1, 3, 0] -> target columns [0, 0, 1, 0, 4]:
    # x = 0 shares column 0 with x = 1 (and x = 3), x = 1 with x = 3 -> both
    # invalid; the nearest valid pixel of each is x = 2 (value 1)
    row = np.array([[[0, 1, 1, 3, 0]]], dtype=np.uint8)
    assert oracle.smp(row, 4).tolist() == [[[1, 1, 1, 3, 0]]]
    # equal distances: the smaller value
    row = np.array([[[7, 2, 2, 9]]], dtype=np.uint8)   # targets [-7, -1, 0, -6]: all valid
    assert oracle.smp(row, 8).tolist() == row.tolist()
    row = np.array([[[5, 1, 9, 0]]], dtype=np.uint8)   # targets [-5, 0, -7, 3]
    assert oracle.smp(row, 10).tolist() == row.tolist()
    row = np.array([[[6, 3, 5, 4, 0]]], dtype=np.uint8)  # targets [-6, -2, -3, -1, 4]
    assert oracle.smp(row, 8).tolist() == row.tolist()
    row = np.array([[[2, 0, 3, 2, 9]]], dtype=np.uint8)  # targets [-2, 1, -1, 1, -5]: x=1 hidden by x=3
    # x = 1 invalid; neighbours x = 0 (2) and x = 2 (3) at distance 1 -> 2
    assert oracle.smp(row, 4).tolist() == [[[2, 2, 3, 2, 9]]]
    # the collision must be within D - 1 columns
    assert oracle.smp(row, 2).tolist() == row.tolist()


def test_smp_brute_force_random_rows():
    rng = np.random.default_rng(7)
    for _ in range(50):
        w, D = int(rng.integers(1, 20)), int(rng.integers(1, 9))
        row = rng.integers(0, D, (1, 1, w)).astype(np.uint8)
        t = np.arange(w) - row[0, 0].astype(int)
        valid = [not any(t[x + k] == t[x] for k in range(1, D) if x + k < w) for x in range(w)]
        exp = row[0, 0].copy()
        for x in range(w):
            if valid[x]:
                continue
            cands = [(abs(x - y), int(row[0, 0, y])) for y in range(w) if valid[y]]
            dmin = min(c[0] for c in cands)
            exp[x] = min(v for dd, v in cands if dd == dmin)
        assert (oracle.smp(row, D)[0, 0] == exp).all()


def test_median_matches_numpy_median():
    rng = np.random.default_rng(8)
    a = rng.integers(0, 256, (2, 9, 13), dtype=np.uint8)
    got = oracle.median3(a)
    pad = np.pad(a, ((0, 0), (1, 1), (1, 1)), mode="edge")
    win = np.stack([pad[:, u:u + 9, t:t + 13] for u in range(3) for t in range(3)], axis=-1)
    assert (got == np.median(win, axis=-1).astype(np.uint8)).all()


def test_sgm_lowers_the_error_on_the_workload_pair():
    # smoothing along paths helps on piecewise-planar scenes: the refined map
    # beats plain winner-take-all against the ground truth at the reduced size
    p = gen_preset("pair256x128")
    lo, cl, cr, d = oracle.match(p.left, p.right, 2, 5, 5, 16)
    _, raw, post = oracle.match_sgm(p.left, p.right, 2, 5, 5, 16, 10, 120)
    gt = (p.gt[::2, ::2] / 2)[:d.shape[1], :d.shape[2]]
    e_wta = np.mean(np.abs(d[0] - gt))
    e_sgm = np.mean(np.abs(raw[0] - gt))
    e_post = np.mean(np.abs(post[0] - gt))
    assert e_sgm < e_wta and e_post < e_sgm


# ---------------------------------------------------------------- ZNCC cost

def _zncc_direct(R, T, i, j, d, rx, ry):
    """Eqs. (1)-(3) written with the window means and deviations, float64."""
    h, w = R.shape
    ys = np.clip(np.arange(i - ry, i + ry + 1), 0, h - 1)
    xr = np.clip(np.arange(j - rx, j + rx + 1), 0, w - 1)
    xt = np.clip(np.arange(j - d - rx, j - d + rx + 1), 0, w - 1)
    r = R[np.ix_(ys, xr)].astype(np.float64)
    t = T[np.ix_(ys, xt)].astype(np.float64)
    dr, dt = r - r.mean(), t - t.mean()
    sr, st = np.sqrt((dr ** 2).sum()), np.sqrt((dt ** 2).sum())
    if sr == 0 or st == 0:
        return 1.0
    return 1.0 - (dr * dt).sum() / (sr * st)


def test_zncc_matches_its_definition():
    rng = np.random.default_rng(9)
    R = rng.integers(0, 256, (9, 14), dtype=np.uint8)
    T = rng.integers(0, 256, (9, 14), dtype=np.uint8)
    T[2:5, 3:8] = 17          # a flat patch: windows inside it have no deviation
    D, ww, wh = 6, 5, 3
    q = oracle.zncc_cost(R, T, D, ww, wh)[0]
    for i in range(9):
        for j in range(14):
            for d in range(D):
                if j - d < 0:
                    assert q[i, j, d] == 64
                    continue
                C = _zncc_direct(R, T, i, j, d, 2, 1)
                x = 32.0 * C + 0.5
                # the two float evaluations may differ only at a rounding tie
                assert q[i, j, d] == np.floor(x) or abs(x - np.round(x)) < 1e-9, (i, j, d, C)


def test_zncc_invariances():
    rng = np.random.default_rng(10)
    R = rng.integers(0, 120, (1, 12, 30), dtype=np.uint8)
    s = 3
    Ts = np.zeros_like(R)
    Ts[:, :, :-s] = R[:, :, s:]                       # the right view is R shifted by s
    T_aff = (2 * Ts.astype(np.int32) + 3).astype(np.uint8)   # and an affine intensity change
    T_neg = (255 - Ts.astype(np.int32)).astype(np.uint8)     # and an inverted one
    for T, expect in ((Ts, 0), (T_aff, 0), (T_neg, 64)):
        q = oracle.zncc_cost(R, T, 8, 5, 5)[0]
        # windows whose clamped targets equal the shifted reference: columns s+2 .. w-3-? inside
        assert (q[:, s + 2:-3, s] == expect).all()
    flat = np.full((1, 6, 10), 9, np.uint8)
    assert (oracle.zncc_cost(flat, R[:, :6, :10], 3, 3, 3)[0][:, 2:, :] == 32).all()


def test_zncc_sgm_recovers_shift():
    rng = np.random.default_rng(12)
    left = rng.integers(0, 256, (1, 40, 64), dtype=np.uint8)
    s = 4
    right = np.zeros_like(left)
    right[:, :, :-s] = left[:, :, s:]
    lo_l, lo_r = oracle.downsample(left, 1), oracle.downsample(right, 1)
    d = oracle.wta(oracle.sgm(oracle.zncc_cost(lo_l, lo_r, 10, 5, 5), 10, 120))
    assert (d[0, 3:-3, s + 3:-3] == s).all()
