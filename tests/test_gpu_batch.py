"""Batched execution: many lattices advanced by one persistent launch.

Every member must equal the oracle's DTr emulation of that lattice alone,
bit for bit, whatever the membership, the per-member MCS counts and rates,
the launch shape (threads, persistent grid, graph capture) and whether the
launch is a graph replay.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (L, D, C, p, q, n_mcs): sizes from one 16-cell domain to 1024-cell domains,
# acceptance draws or not, different MCS counts (different phases of the queue)
MIX = [
    (64, 16, 8, 1.0, 0.0, 3),
    (128, 32, 8, 0.5, 0.5, 5),
    (64, 8, 4, 0.95, 0.05, 2),
    (128, 64, 8, 1.0, 0.0, 4),
    (256, 128, 8, 0.7, 0.2, 1),
    (64, 32, 2, 0.0, 1.0, 3),
]


class Mirror:
    """The oracle's copy of one member."""

    def __init__(self, orc, L, D, C, scheme, p, q, stream):
        self.emu = orc.Emu(L=L, Dx=D, Dy=D, Cx=C, Cy=C, scheme=scheme, p=p, q=q, seed=7, stream=stream)
        self.s = orc.init_flat(L)
        self.m = 0

    def run(self, n):
        for _ in range(n):
            self.emu.mcs(self.s, self.m)
            self.m += 1


def make_batch(okpz, orc, scheme, mix=MIX):
    b = okpz.Batch()
    lats, mirrors = [], []
    for i, (L, D, C, p, q, n) in enumerate(mix):
        lats.append(b.lattice(L, D, D, C, C, scheme, seed=7, stream=100 + i))
        mirrors.append(Mirror(orc, L, D, C, scheme, p, q, 100 + i))
    return b, lats, mirrors


def run_both(b, lats, mirrors, mix, ns):
    b.run([n for n in ns], [m[3] for m in mix], [m[4] for m in mix])
    b.sync()
    for lat, mir, n in zip(lats, mirrors, ns):
        mir.run(n)
        assert lat.mcs == mir.m
        assert np.array_equal(lat.sites(), mir.s), (lat.L, mir.m)


@pytest.mark.parametrize("scheme", [0, 1, 2], ids=["DT", "DB", "DTr"])
def test_batch_matches_oracle(okpz, orc, scheme):
    b, lats, mirrors = make_batch(okpz, orc, scheme)
    ns = [m[5] for m in MIX]
    run_both(b, lats, mirrors, MIX, ns)          # first launch: capture
    run_both(b, lats, mirrors, MIX, ns)          # same tables: graph replay
    run_both(b, lats, mirrors, MIX, [1, 0, 2, 0, 1, 3])  # some members idle
    b.close()


@pytest.mark.parametrize("threads,grid,graph", [(64, 0, True), (128, 1, False), (256, 3, True), (256, 0, False),
                                                (512, 0, True), (512, 2, False)])
def test_batch_launch_shape_does_not_change_results(okpz, orc, threads, grid, graph):
    b, lats, mirrors = make_batch(okpz, orc, 1)
    b.config(threads, grid, graph)
    run_both(b, lats, mirrors, MIX, [2, 3, 1, 2, 1, 2])
    run_both(b, lats, mirrors, MIX, [2, 3, 1, 2, 1, 2])
    b.close()


def test_batch_membership_and_outside_runs(okpz, orc):
    b, lats, mirrors = make_batch(okpz, orc, 0, MIX[:4])
    mix = MIX[:4]
    run_both(b, lats, mirrors, mix, [1, 1, 1, 1])
    # a member run alone between batch runs (the batch re-reads its MCS count)
    lats[1].run(2, mix[1][3], mix[1][4])
    mirrors[1].run(2)
    run_both(b, lats, mirrors, mix, [1, 1, 1, 1])
    # remove a member, add a new one into the freed slot
    b.remove(lats[2].slot)
    assert b.size == 4
    newlat = b.lattice(128, 16, 16, 8, 8, 0, seed=7, stream=300)
    assert newlat.slot == 2
    newmir = Mirror(orc, 128, 16, 8, 0, 1.0, 0.0, 300)
    mix2 = [mix[0], mix[1], (128, 16, 8, 1.0, 0.0, 1), mix[3]]
    lats2 = [lats[0], lats[1], newlat, lats[3]]
    mirrors2 = [mirrors[0], mirrors[1], newmir, mirrors[3]]
    run_both(b, lats2, mirrors2, mix2, [2, 1, 3, 1])
    # the removed lattice still works on its own
    lats[2].run(1, mix[2][3], mix[2][4])
    mirrors[2].run(1)
    assert np.array_equal(lats[2].sites(), mirrors[2].s)
    # measurement of a member after batch runs
    mo = lats[0].measure()
    assert mo["w2"] == orc.w2(mirrors[0].s)
    b.close()


def test_batch_equals_plain_runs(okpz):
    """A slice of the batched workload (uneven L, D = min(256, L/2), (1,0) and
    (1/2,1/2)): every member equals the same lattice run alone with okpz_run."""
    from workloads import batched_composition

    comp = batched_composition(n=24, seed=1)
    b = okpz.Batch()
    batched, alone = [], []
    for c in comp:
        batched.append(b.lattice(c.L, c.Dx, c.Dy, c.Cx, c.Cy, c.scheme, seed=1, stream=c.stream))
        alone.append(okpz.Lattice(c.L, c.Dx, c.Dy, c.Cx, c.Cy, c.scheme, seed=1, stream=c.stream))
    b.run([3] * len(comp), [c.p for c in comp], [c.q for c in comp])
    b.run([2] * len(comp), [c.p for c in comp], [c.q for c in comp])
    b.sync()
    for lat, c in zip(alone, comp):
        lat.run(5, c.p, c.q)
    for x, y in zip(batched, alone):
        assert x.mcs == y.mcs == 5
        assert np.array_equal(x.words(), y.words())
    b.close()


# Long runs of lone lattices and pairs, where the steps of one lattice overlap
# most (few tiles per step): (L, D, C, scheme, p, q, MCS, members).  D from 8
# (footprint margins span 3 tiles more: 31 // 8) to 256 (one tile either side).
LONG = [
    (2048, 256, 8, 1, 0.95, 0.05, 300, 1),
    (1024, 256, 8, 0, 1.0, 0.0, 400, 2),
    (512, 64, 8, 2, 0.7, 0.2, 300, 1),
    (512, 16, 8, 1, 1.0, 0.0, 200, 1),
    (256, 8, 4, 0, 0.5, 0.5, 300, 2),
    (1024, 32, 8, 1, 0.95, 0.05, 200, 3),
]


@pytest.mark.parametrize("case", LONG, ids=lambda c: "L%d_D%d_C%d_s%d_n%d" % (c[0], c[1], c[2], c[3], c[7]))
def test_batch_long_runs_equal_plain(okpz, case):
    """The steps of one lattice overlap across tiles inside a batch launch
    (each tile waits only for the tiles whose memory words it can share); over
    hundreds of MCS, with random origins that move the tiling every MCS, every
    member still equals the lattice run alone step by step."""
    L, D, C, scheme, p, q, mcs, n = case
    b = okpz.Batch()
    batched = [b.lattice(L, D, D, C, C, scheme, seed=3, stream=40 + i) for i in range(n)]
    alone = [okpz.Lattice(L, D, D, C, C, scheme, seed=3, stream=40 + i) for i in range(n)]
    b.run([mcs] * n, p, q)
    b.sync()
    for lat in alone:
        lat.run(mcs, p, q)
    for x, y in zip(batched, alone):
        assert x.mcs == y.mcs == mcs
        assert np.array_equal(x.words(), y.words())
    b.close()
    for lat in batched + alone:
        lat.close()


def test_batch_rejects_bad_arguments(okpz):
    b = okpz.Batch()
    a = b.lattice(64, 16, 16, 8, 8, 0)
    with pytest.raises(okpz.OkpzError):
        b.add(a)                                   # already a member
    other = okpz.Lattice(64, 16, 16, 8, 8, 0)      # null stream
    with pytest.raises(okpz.OkpzError):
        b.add(other)
    with pytest.raises(okpz.OkpzError):
        b.lattice(64, 16, 16, 8, 8, 1)             # another block scheme
    with pytest.raises(okpz.OkpzError):
        b.run([1], [1.5], [0.0])                   # p outside [0, 1]
    with pytest.raises(okpz.OkpzError):
        b.config(96, 0, True)
    b.remove(a.slot)
    with pytest.raises(okpz.OkpzError):
        b.remove(a.slot)
    assert b.size == 0
    b.run([], [], [])                              # nothing to do
    b.close()
    other.close()


@pytest.mark.parametrize("threads", [64, 128, 0])
def test_batch_db_column_sweep(okpz, orc, threads):
    """DB lattices whose domains all hold lanes x cells-per-lane cells take the
    column-mapped sweep (64 or 128 lanes here; the default width takes the
    generic one): same results."""
    mix = [(128, 64, 4, 0.95, 0.05, 3), (256, 64, 4, 1.0, 0.0, 2), (128, 64, 4, 0.6, 0.4, 4),
           (256, 128, 8, 0.8, 0.3, 2)]
    b, lats, mirrors = make_batch(okpz, orc, 1, mix)
    b.config(threads, 0, True)
    run_both(b, lats, mirrors, mix, [m[5] for m in mix])
    run_both(b, lats, mirrors, mix, [1, 2, 1, 1])
    b.close()


@pytest.mark.parametrize("threads", [512, 256])
def test_batch_db_column_sweep_1024_cells(okpz, orc, threads):
    """1024-cell DB domains (D = 256, TC = 1,1) in the column-mapped sweep with
    512 lanes x 2 cells and 256 lanes x 4 cells: the oracle's results."""
    mix = [(512, 256, 8, 0.95, 0.05, 2), (512, 256, 8, 1.0, 0.0, 3)]
    b, lats, mirrors = make_batch(okpz, orc, 1, mix)
    b.config(threads, 0, True)
    run_both(b, lats, mirrors, mix, [m[5] for m in mix])
    b.close()


ROW_MIXES = {
    # every member DB with square 256- or 128-site domains of 8 x 8-site cells
    # and one lane-field width: the batch kernel's row-paired sweep
    "D256_accept": [(512, 256, 8, 0.95, 0.05, 3), (1024, 256, 8, 0.7, 0.3, 2), (512, 256, 8, 0.5, 0.5, 4)],
    "D256_p1": [(512, 256, 8, 1.0, 0.0, 3), (1024, 256, 8, 0.0, 1.0, 2)],
    "D128_accept": [(256, 128, 8, 0.9, 0.1, 3), (512, 128, 8, 0.6, 0.4, 2), (256, 128, 8, 0.999, 0.001, 5)],
}


@pytest.mark.parametrize("threads", [0, 256, 512])
@pytest.mark.parametrize("mix", sorted(ROW_MIXES))
def test_batch_db_row_sweep(okpz, orc, mix, threads):
    """Batches whose members all take the row-paired DB sweep (two cells per
    lane, whatever width is configured): the oracle's results, including a
    second run that replays the captured launch."""
    m = ROW_MIXES[mix]
    b, lats, mirrors = make_batch(okpz, orc, 1, m)
    b.config(threads, 0, True)
    run_both(b, lats, mirrors, m, [x[5] for x in m])
    run_both(b, lats, mirrors, m, [x[5] for x in m])
    b.close()


DT_ROW_MIXES = {
    # DT / DTr members with square 128- and 256-site domains of 8 x 8-site
    # cells, with and without acceptance prefixes in one batch (lane fields of
    # 16 and 4 bits): the batch kernel's row-paired DT sweep, each item for its
    # own domain size and rates; 128-site members leave lanes idle
    "mixed": [(512, 256, 8, 1.0, 0.0, 3), (256, 128, 8, 0.5, 0.5, 4), (1024, 256, 8, 0.95, 0.05, 2),
              (256, 128, 8, 1.0, 0.0, 5), (512, 256, 8, 0.3, 0.9, 2)],
    "D128": [(256, 128, 8, 0.95, 0.05, 3), (512, 128, 8, 1.0, 0.0, 2)],
}


@pytest.mark.parametrize("threads", [0, 256, 512])
@pytest.mark.parametrize("scheme", [0, 2], ids=["DT", "DTr"])
@pytest.mark.parametrize("mix", sorted(DT_ROW_MIXES))
def test_batch_dt_row_sweep(okpz, orc, mix, scheme, threads):
    """Batches whose members all take the row-paired DT / DTr sweep: the
    oracle's results, including a second run that replays the captured
    launch."""
    m = DT_ROW_MIXES[mix]
    b, lats, mirrors = make_batch(okpz, orc, scheme, m)
    b.config(threads, 0, True)
    run_both(b, lats, mirrors, m, [x[5] for x in m])
    run_both(b, lats, mirrors, m, [x[5] for x in m])
    b.close()
