"""GPU checks at the full single-lattice size L = 2^17 (2^34 sites, 4 GiB packed),
in the launch configuration the benchmark times (256x256 domains, TC=1,1,
DTrDB, p=0.95, q=0.05).

* lattice: after one MCS from flat, a 3072x3072 window (wrapping the periodic
  boundary) equals the oracle's window emulation on every site the oracle can
  determine (domains wholly inside the window);
* moments: flat state and a flat state with a local bump written in, against
  closed forms (flat moments analytic; the bump's contribution to the height
  moments, C_h and C_s from the oracle's values on the bumped piece);
* invariants: particle conservation per sampled row and column, plaquette
  closure on sampled windows, C_h(s,s) = W^2(s), after several MCS.
"""
from fractions import Fraction

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

L = 1 << 17
D, C = 256, 8
P, Q = 0.95, 0.05


@pytest.fixture(scope="module")
def big(okpz):
    lat = okpz.Lattice(L, D, D, C, C, okpz.BLOCK_DB, seed=1, stream=0)
    yield lat
    lat.close()


def flat_moments():
    n = L * L
    return {"n_even": n // 2, "n_odd": n // 2, "s1_even": 0, "s1_odd": n // 2, "s2_even": 0,
            "s2_odd": n // 2}


def w2_exact(mo):
    n = mo["n_even"] + mo["n_odd"]
    s1 = mo["s1_even"] + mo["s1_odd"]
    s2 = mo["s2_even"] + mo["s2_odd"]
    return float(Fraction(n * s2 - s1 * s1, n * n))


def test_flat_moments_closed_form(big):
    big.init_flat()
    mo = big.measure()
    for k, v in flat_moments().items():
        assert mo[k] == v, k
    assert mo["w2"] == 0.25 and mo["w2_sub"] == 0.0


def test_local_bump_moments_and_autocorr(big, orc):
    # build a bump on a 64x64 flat piece with the oracle's rule, away from the
    # piece's edges, and write it into the flat lattice at an even-parity corner
    piece = orc.init_flat(64)
    rng = np.random.default_rng(9)
    for _ in range(6000):
        x, y = int(rng.integers(8, 56)), int(rng.integers(8, 56))
        orc.attempt(piece, x, y, True, rng.random() < 0.3)
    flat_piece = orc.init_flat(64)
    assert orc.check_state(piece) == 0
    hb = orc.heights(piece)
    hf = orc.heights(flat_piece)
    assert hb[0, 0] == hf[0, 0] == 0 and np.array_equal(hb[:4], hf[:4])
    x0, y0 = L - 1000, 70000  # x0 + y0 even: the flat pattern matches the piece's
    big.init_flat()
    big.snapshot()
    big.set_window(x0, y0, piece)
    assert np.array_equal(big.window(x0, y0, 64, 64), piece)
    exp = flat_moments()
    par = ((np.add.outer(np.arange(64), np.arange(64))) & 1).astype(bool)  # same parity as global
    for cls, name in ((False, "even"), (True, "odd")):
        sel = par == cls
        exp["s1_" + name] += int((hb[sel] - hf[sel]).sum())
        exp["s2_" + name] += int((hb[sel] ** 2 - hf[sel] ** 2).sum())
    mo = big.measure()
    for k, v in exp.items():
        assert mo[k] == v, k
    assert mo["w2"] == w2_exact(exp)
    # C_h(t, s) with s = the flat state (snapshot taken before the bump was
    # written) and t = the bumped state: sum h_t h_s = S2_flat + sum h_f (h_b - h_f)
    ac = big.autocorr()
    n = L * L
    s_ts = n // 2 + int((hf * (hb - hf)).sum())
    s1_t = exp["s1_even"] + exp["s1_odd"]
    s1_s = n // 2
    assert ac["s_ts"] == s_ts and ac["s1_t"] == s1_t and ac["s1_s"] == s1_s
    assert ac["c_h"] == float(Fraction(n * s_ts - s1_t * s1_s, n * n))
    # C_s: the flat lattice overlaps itself in L^2 slope variables; inside the
    # bumped piece the overlap is the piece's own overlap with flat
    ov = n - orc.slope_overlap(flat_piece, flat_piece) + orc.slope_overlap(piece, flat_piece)
    assert ac["overlap"] == ov
    assert ac["c_s"] == float(Fraction(ov, 2 * n) - Fraction(1, 4))


def test_one_mcs_window_parity(big, orc):
    big.init_flat()
    big.run(1, P, Q)
    window = (L - 1500, 2000, 3072, 3072)  # wraps in x
    wx0, wy0, W, H = window
    got = big.window(wx0, wy0, W, H)
    emu = orc.Emu(L=L, Dx=D, Dy=D, Cx=C, Cy=C, scheme=orc.DB, p=P, q=Q, seed=1, stream=0)
    ref, valid = orc.init_flat_window(L, window)
    emu.mcs_window(ref, valid, window, 0)
    v = valid.astype(bool)
    assert v.sum() > 0.3 * W * H
    assert np.array_equal(got[v], ref[v])
    # sites the oracle could not determine were still updated by the GPU run:
    # the window is not left flat there
    flat, _ = orc.init_flat_window(L, window)
    assert (got[~v] != flat[~v]).any()


def test_invariants_after_several_mcs(big):
    big.init_flat()
    big.run(3, P, Q)
    big.snapshot()
    mo = big.measure()
    ac = big.autocorr()
    assert ac["c_h"] == mo["w2"] and ac["s_ts"] == mo["s2_even"] + mo["s2_odd"]
    assert ac["c_s"] == 0.25 and ac["overlap"] == L * L
    assert mo["w2"] > 0.25
    rng = np.random.default_rng(3)
    for y in rng.integers(0, L, 3):
        row = big.window(0, int(y), L, 1)[0]
        assert int((row & 1).sum()) == L // 2
    for x in rng.integers(0, L, 3):
        col = big.window(int(x), 0, 1, L)[:, 0]
        assert int(((col >> 1) & 1).sum()) == L // 2
    for _ in range(3):
        x0, y0 = (int(v) for v in rng.integers(0, L, 2))
        w = big.window(x0, y0, 512, 512).astype(np.int64)
        sx, sy = w & 1, (w >> 1) & 1
        # sx[x,y-1] + sy[x,y] == sy[x-1,y] + sx[x,y] inside the window
        assert np.array_equal(sx[:-1, 1:] + sy[1:, 1:], sy[1:, :-1] + sx[1:, 1:])
    big.run(1, P, Q)
    assert big.mcs == 4
