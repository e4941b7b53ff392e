"""Pin the oracle's update rule on the 8x8 torus by brute force.

The 4x4 torus is enumerated whole (test_oracle_rule.py); the 8x8 torus has too
many surfaces for that, so valid 8x8 surfaces are generated here without the
oracle -- random walks of the octahedron move written on heights (Sec. 2.1:
deposition raises a local minimum by 2, removal lowers a local maximum by 2)
from the flat zig-zag surface, with drifts from growth to etching -- until
every site of the torus (interior, the wrap column x = 7 and the wrap row
y = 7 included) has been seen in all sixteen slope patterns of its four
links, the local minimum and maximum among them.  On every collected surface
the oracle's bit rule must agree with the height rule at every site and for
every acceptance outcome.
"""
import numpy as np

from l4_states import height_rule, slopes_from_heights

L = 8


def _flat_heights():
    return (np.add.outer(np.arange(L), np.arange(L)) & 1).astype(np.int64)


def _local_pattern(s, x, y):
    """(sx(x,y), sx(x+1,y), sy(x,y), sy(x,y+1)) as a 4-bit number."""
    a = s[y, x] & 1
    b = s[y, (x + 1) % L] & 1
    c = (s[y, x] >> 1) & 1
    d = (s[(y + 1) % L, x] >> 1) & 1
    return int(a) << 3 | int(b) << 2 | int(c) << 1 | int(d)


def _surfaces():
    rng = np.random.default_rng(88)
    seen = np.zeros((L, L, 16), dtype=bool)
    states = []
    while not seen.all() and len(states) < 4000:
        h = _flat_heights()
        p = rng.uniform(0.05, 0.95)
        steps = int(rng.integers(1, 400))
        for _ in range(steps):
            x, y = int(rng.integers(0, L)), int(rng.integers(0, L))
            h = height_rule(h, x, y, rng.random() < p, rng.random() < 1.0 - p)
        s = slopes_from_heights(h)
        for y in range(L):
            for x in range(L):
                seen[y, x, _local_pattern(s, x, y)] = True
        states.append(h)
    assert seen.all(), "the random walks did not reach every local pattern at every site"
    return states


def test_bit_rule_equals_height_rule_8x8(orc):
    states = _surfaces()
    assert len(states) >= 16
    flips = 0
    for h in states:
        s = slopes_from_heights(h)
        assert orc.check_state(s) == 0
        for y in range(L):
            for x in range(L):
                for dep, rem in ((True, False), (False, True), (True, True), (False, False)):
                    t = s.copy()
                    ret = orc.attempt(t, x, y, dep, rem)
                    g = height_rule(h, x, y, dep, rem)
                    assert np.array_equal(t, slopes_from_heights(g)), (x, y, dep, rem)
                    dh = (g[y, x] - g[0, 0]) - (h[y, x] - h[0, 0])
                    if (x, y) != (0, 0):
                        assert ret == dh // 2
                    flips += ret != 0
    assert flips > 0


def test_minimum_and_maximum_patterns_8x8(orc):
    """At every site the local minimum (0,1,0,1) deposits only when allowed and
    the local maximum (1,0,1,0) is removed only when allowed; no other pattern
    changes anything."""
    for h in _surfaces()[:200]:
        s = slopes_from_heights(h)
        for y in range(L):
            for x in range(L):
                pat = _local_pattern(s, x, y)
                for dep, rem in ((True, False), (False, True)):
                    t = s.copy()
                    orc.attempt(t, x, y, dep, rem)
                    changed = not np.array_equal(t, s)
                    assert changed == ((pat == 0b0101 and dep) or (pat == 0b1010 and rem)), (x, y, pat)
