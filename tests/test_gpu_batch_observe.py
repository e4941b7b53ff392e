"""Batched observables: the moments, C_h and C_s of every member of a batch
from three launches, against the oracle's exact integers for each member's
state (and the oracle's own DTr emulation of that member), plus the measured
series entry point.

Members of different L (64 .. 512, one to 32 bands of blocks per lattice row)
share each launch, so the band-to-member mapping, the per-member reduction and
the snapshot copies (partial and whole 16-KiB chunks) are all exercised.
"""
import numpy as np
import pytest

from test_gpu_batch import Mirror

pytestmark = pytest.mark.gpu

# (L, D, C, p, q, n_mcs)
MIX = [
    (64, 16, 8, 1.0, 0.0, 3),
    (512, 64, 8, 0.5, 0.5, 2),
    (128, 32, 8, 0.95, 0.05, 5),
    (256, 128, 8, 0.7, 0.2, 1),
    (64, 8, 4, 0.0, 1.0, 4),
]


def check_member(orc, mo, co, st, ss, t, s):
    ref = orc.moments(st)
    for k in ("n_even", "n_odd", "s1_even", "s1_odd", "s2_even", "s2_odd"):
        assert mo[k] == ref[k], k
    assert mo["mcs"] == t
    assert mo["w2"] == orc.w2_from_moments(ref)
    assert mo["w2_sub"] == orc.w2_sub_from_moments(ref)
    if co is None:
        return
    assert co["t"] == t and co["s"] == s
    assert co["s_ts"] == orc.cross(st, ss)
    ms = orc.moments(ss)
    assert co["s1_s"] == ms["s1_even"] + ms["s1_odd"]
    assert co["s1_t"] == ref["s1_even"] + ref["s1_odd"]
    assert co["c_h"] == orc.c_h(st, ss)
    assert co["overlap"] == orc.slope_overlap(st, ss)
    assert co["c_s"] == orc.c_s(st, ss)


@pytest.mark.parametrize("scheme", [0, 1], ids=["DT", "DB"])
def test_batch_observe_matches_oracle(okpz, orc, scheme):
    b = okpz.Batch()
    lats, mirs = [], []
    for i, (L, D, C, p, q, n) in enumerate(MIX):
        lats.append(b.lattice(L, D, D, C, C, scheme, seed=7, stream=200 + i))
        mirs.append(Mirror(orc, L, D, C, scheme, p, q, 200 + i))
    p = [m[3] for m in MIX]
    q = [m[4] for m in MIX]
    ns = [m[5] for m in MIX]
    # at t = 0 the flat state: W^2 = 1/4, W^2_sub = 0
    obs = b.observe()
    for s, lat in enumerate(lats):
        assert obs[s][0]["w2"] == 0.25 and obs[s][0]["w2_sub"] == 0.0
    b.run(ns, p, q)
    for mir, n in zip(mirs, ns):
        mir.run(n)
    b.snapshot()
    snaps = [mir.s.copy() for mir in mirs]
    svals = [mir.m for mir in mirs]
    b.run(ns[::-1], p, q)
    for mir, n in zip(mirs, ns[::-1]):
        mir.run(n)
    obs = b.observe(with_autocorr=True)
    for s, (lat, mir) in enumerate(zip(lats, mirs)):
        assert np.array_equal(lat.sites(), mir.s), lat.L
        mo, co = obs[s]
        check_member(orc, mo, co, mir.s, snaps[s], mir.m, svals[s])
        # the single-lattice pass gives the same values
        m1, c1 = lat.observe(with_autocorr=True)
        assert m1 == mo and c1 == co
    b.close()
    for lat in lats:
        lat.close()


def test_batch_series_matches_oracle_and_free_slots(okpz, orc):
    b = okpz.Batch()
    lats, mirs = [], []
    for i, (L, D, C, p, q, n) in enumerate(MIX[:4]):
        lats.append(b.lattice(L, D, D, C, C, 1, seed=7, stream=300 + i))
        mirs.append(Mirror(orc, L, D, C, 1, p, q, 300 + i))
    # a free slot inside the table
    b.remove(1)
    live = [0, 2, 3]
    p = {s: MIX[s][3] for s in live}
    q = {s: MIX[s][4] for s in live}
    b.run({s: 2 for s in live}, p, q)
    for s in live:
        mirs[s].run(2)
    b.snapshot()
    snaps = {s: mirs[s].s.copy() for s in live}
    times = [0, 1, 3, 3, 6]
    out = b.series(times, p, q, with_autocorr=True)
    assert len(out) == len(times)
    t_prev = 0
    for i, t in enumerate(times):
        assert sorted(out[i]) == live
        for s in live:
            mirs[s].run(t - t_prev)
            mo, co = out[i][s]
            check_member(orc, mo, co, mirs[s].s, snaps[s], 2 + t, 2)
        t_prev = t
    for s in live:
        assert np.array_equal(lats[s].sites(), mirs[s].s)
    b.close()
    for lat in lats:
        lat.close()


def test_batch_observe_errors(okpz):
    b = okpz.Batch()
    lats = [b.lattice(64, 16, 16, 8, 8, 0, seed=1, stream=i) for i in range(2)]
    with pytest.raises(okpz.OkpzError) as e:
        b.observe(with_autocorr=True)  # no snapshot yet
    assert e.value.status == okpz.ESTATE
    with pytest.raises(okpz.OkpzError) as e:
        b.series([2, 1], 1.0, 0.0)  # times must not decrease
    assert e.value.status == okpz.EINVAL
    assert all(lat.mcs == 0 for lat in lats)  # nothing ran
    with pytest.raises(okpz.OkpzError) as e:
        b.series([1], 1.5, 0.0)
    assert e.value.status == okpz.EINVAL
    # an empty series and an empty batch are fine
    assert b.series([], 1.0, 0.0) == []
    e2 = okpz.Batch()
    assert e2.observe() == {}
    e2.snapshot()
    e2.close()
    b.close()
    for lat in lats:
        lat.close()


def test_batch_observe_large_member(okpz, orc):
    """A 2048 lattice beside a 64 one: 512 bands and a 64-chunk snapshot copy
    for one member, one band row and a partial chunk for the other."""
    b = okpz.Batch()
    cfg = [(2048, 256, 8, 0.95, 0.05), (64, 16, 8, 1.0, 0.0)]
    lats = [b.lattice(L, D, D, C, C, 1, seed=7, stream=i + 1) for i, (L, D, C, _, _) in enumerate(cfg)]
    mirs = [Mirror(orc, L, D, C, 1, p, q, i + 1) for i, (L, D, C, p, q) in enumerate(cfg)]
    p = [c[3] for c in cfg]
    q = [c[4] for c in cfg]
    b.run([3, 3], p, q)
    for m in mirs:
        m.run(3)
    b.snapshot()
    snaps = [m.s.copy() for m in mirs]
    b.run([2, 2], p, q)
    for m in mirs:
        m.run(2)
    obs = b.observe(with_autocorr=True)
    for s, (lat, mir) in enumerate(zip(lats, mirs)):
        assert np.array_equal(lat.sites(), mir.s)
        check_member(orc, obs[s][0], obs[s][1], mir.s, snaps[s], 5, 3)
    b.close()
    for lat in lats:
        lat.close()
