"""Pin the oracle's update rule, state checks and heights by brute force.

The reference for the rule is the octahedron move written on heights
(Sec. 2.1: deposition on a local minimum raises it by 2, removal on a local
maximum lowers it by 2), applied to every state of the 4x4 torus.  The bit
rule in the oracle (Kawasaki dimer exchange on slopes) must agree on every
state, site and acceptance outcome.
"""
import numpy as np
import pytest

from l4_states import StateSpace, height_rule, slopes_from_heights, w2_of_heights, w2_sub_of_heights


@pytest.fixture(scope="module")
def space():
    return StateSpace(4)


def test_state_count(space):
    # every height function on the 4x4 torus with h(0,0)=0
    assert len(space) == 990


def test_bit_rule_equals_height_rule(orc, space):
    mismatches = 0
    for h, s in zip(space.heights, space.slopes):
        for y in range(4):
            for x in range(4):
                for dep, rem in ((True, False), (False, True), (True, True), (False, False)):
                    t = s.copy()
                    ret = orc.attempt(t, x, y, dep, rem)
                    g = height_rule(h, x, y, dep, rem)
                    expect = slopes_from_heights(g)
                    if not np.array_equal(t, expect):
                        mismatches += 1
                    dh = (g[y, x] - g[0, 0]) - (h[y, x] - h[0, 0]) if (x, y) != (0, 0) else 0
                    if (x, y) != (0, 0):
                        assert ret == dh // 2
    assert mismatches == 0


def test_valid_states_pass_check(orc, space):
    for s in space.slopes:
        assert orc.check_state(s) == 0


def test_invalid_states_fail_check(orc, space):
    rng = np.random.default_rng(5)
    for s in space.slopes[::37]:
        for _ in range(4):
            t = s.copy()
            y, x, b = rng.integers(0, 4), rng.integers(0, 4), rng.integers(0, 2)
            t[y, x] ^= np.uint8(1 << b)
            assert orc.check_state(t) != 0


def test_all_states_reachable_from_flat(orc, space):
    start = space.flat_index()
    seen = {start}
    frontier = [start]
    while frontier:
        nxt = []
        for i in frontier:
            for y in range(4):
                for x in range(4):
                    for dep, rem in ((True, False), (False, True)):
                        t = space.slopes[i].copy()
                        orc.attempt(t, x, y, dep, rem)
                        j = space.index[t.tobytes()]
                        if j not in seen:
                            seen.add(j)
                            nxt.append(j)
        frontier = nxt
    assert len(seen) == 990


def test_heights_match_enumerated(orc, space):
    for h, s in zip(space.heights, space.slopes):
        assert np.array_equal(orc.heights(s), h)


def test_heights_track_net_deposits(orc):
    # heights from slopes equal flat heights + 2 * (net deposits per site),
    # up to one global constant, along a long random sequence of attempts
    L = 16
    rng = np.random.default_rng(11)
    s = orc.init_flat(L)
    net = np.zeros((L, L), dtype=np.int64)
    flat_h = (np.add.outer(np.arange(L), np.arange(L)) & 1).astype(np.int64)
    for _ in range(20000):
        x, y = int(rng.integers(0, L)), int(rng.integers(0, L))
        net[y, x] += orc.attempt(s, x, y, rng.random() < 0.7, rng.random() < 0.4)
    h = orc.heights(s)
    expect = flat_h + 2 * net
    d = h - expect
    assert np.all(d == d[0, 0])
    assert orc.check_state(s) == 0


def test_conservation_along_dynamics(orc):
    L = 16
    rng = np.random.default_rng(3)
    s = orc.init_flat(L)
    for _ in range(5000):
        orc.attempt(s, int(rng.integers(0, L)), int(rng.integers(0, L)), True, rng.random() < 0.5)
        assert np.all((s & 1).sum(axis=1) == L // 2)
        assert np.all(((s >> 1) & 1).sum(axis=0) == L // 2)
    assert orc.check_state(s) == 0


def test_flat_moments_closed_form(orc):
    for L in (4, 8, 64, 256):
        s = orc.init_flat(L)
        mo = orc.moments(s)
        n = L * L
        assert mo == {"n_even": n // 2, "n_odd": n // 2, "s1_even": 0, "s1_odd": n // 2,
                      "s2_even": 0, "s2_odd": n // 2}
        assert orc.w2_from_moments(mo) == 0.25
        assert orc.w2_sub_from_moments(mo) == 0.0


def test_single_deposit_closed_form(orc):
    L = 32
    s = orc.init_flat(L)
    x, y = 6, 10  # even site (x+y even): h = 0, all neighbours at 1 -> local minimum
    assert orc.attempt(s, x, y, True, False) == 1
    mo = orc.moments(s)
    n = L * L
    assert mo["s1_even"] == 2 and mo["s2_even"] == 4
    assert mo["s1_odd"] == n // 2 and mo["s2_odd"] == n // 2
    s1, s2 = n // 2 + 2, n // 2 + 4
    assert orc.w2(s) == (n * s2 - s1 * s1) / (n * n)
    # C_h(t,s) between the perturbed state and the flat start
    f = orc.init_flat(L)
    assert orc.cross(s, f) == n // 2  # sum h_t h_s: only odd sites (h=1 in both) contribute
    assert orc.c_h(s, f) == (n * (n // 2) - s1 * (n // 2)) / (n * n)


def test_w2_and_w2sub_on_all_states(orc, space):
    for h, s in zip(space.heights, space.slopes):
        mo = orc.moments(s)
        w2, w2s = orc.w2_from_moments(mo), orc.w2_sub_from_moments(mo)
        assert abs(w2 - w2_of_heights(h)) < 1e-15
        assert abs(w2s - w2_sub_of_heights(h)) < 1e-15
        assert -1e-15 <= w2 - w2s <= 0.25 + 1e-15


def test_autocorr_equal_times_is_w2(orc):
    L = 32
    rng = np.random.default_rng(2)
    s = orc.init_flat(L)
    for _ in range(3000):
        orc.attempt(s, int(rng.integers(0, L)), int(rng.integers(0, L)), True, False)
    assert orc.c_h(s, s) == orc.w2(s)


def test_slope_autocorr_definition_on_all_states(orc, space):
    """C_s (Sec. 2.1) from the oracle's overlap count equals the definition
    <n_t n_s> - <n_t><n_s> evaluated on slopes derived from enumerated heights
    (means taken from the data, not assumed), for every 4x4 state against
    several references; every state has <n> = 1/2 and C_s(s,s) = 1/4."""
    refs = [space.slopes[i] for i in (0, 17, 333, 640, 989)]
    for s in space.slopes:
        n_s = np.concatenate([(s & 1).ravel(), ((s >> 1) & 1).ravel()]).astype(np.int64)
        assert n_s.mean() == 0.5
        assert orc.c_s(s, s) == 0.25
        for r in refs:
            n_r = np.concatenate([(r & 1).ravel(), ((r >> 1) & 1).ravel()]).astype(np.int64)
            want = (n_s * n_r).mean() - n_s.mean() * n_r.mean()
            assert orc.c_s(s, r) == want == orc.c_s(r, s)


def test_slope_autocorr_closed_forms(orc):
    for L in (4, 16, 64):
        f = orc.init_flat(L)
        # the flat state of opposite phase has every slope reversed
        g = (f ^ 3).astype(np.uint8)
        assert orc.check_state(g) == 0
        assert orc.c_s(f, g) == -0.25
        # one deposit flips four slopes: two 1 -> 0, two 0 -> 1
        s = f.copy()
        assert orc.attempt(s, 2, 0, True, False) == 1
        assert orc.slope_overlap(s, f) == L * L - 2
        assert orc.c_s(s, f) == 0.25 - 1.0 / (L * L)
