"""Parity of the row-paired DB device step (square 128- and 256-site domains,
8 x 8-site cells, two or four cells per lane) with the oracle's DTr
emulation, bit for bit after every MCS: every workgroup shape that selects
it, rates with and without acceptance prefixes, rates whose thresholds tie
often (the 32-bit tie-break draw decides), and both stochastic directions."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (Dx, threads): 256-site domains have 1024 cells (512 lanes: 2 per lane,
# 256 lanes: 4); 128-site domains have 256 cells (128 lanes: 2, 64 lanes: 4)
SHAPES = [(256, 512), (256, 256), (128, 128), (128, 64)]
RATES = [(1.0, 0.0), (0.95, 0.05), (0.5, 0.5), (0.3, 0.9), (0.0, 1.0), (1.0, 1.0),
         # thresholds with nonzero low words: P = 0.9990234375 + 2^-20 ties at prefix 1023
         (1023 / 1024 + 2.0 ** -20, 1 / 1024 + 2.0 ** -21)]


def _run(okpz, orc, L, D, threads, p, q, n_mcs, stream):
    e = orc.Emu(L=L, Dx=D, Dy=D, Cx=8, Cy=8, scheme=orc.DB, p=p, q=q, seed=11, stream=stream)
    ref = orc.init_flat(L)
    with okpz.Lattice(L, D, D, 8, 8, okpz.BLOCK_DB, 11, stream) as lat:
        lat.set_threads(threads)
        for m in range(n_mcs):
            print("db_rows: L=%d D=%d threads=%d p=%r q=%r MCS %d" % (L, D, threads, p, q, m), flush=True)
            lat.run(1, p, q)
            e.mcs(ref, m)
            got = lat.sites()
            if not np.array_equal(got, ref):
                bad = np.argwhere(got != ref)
                raise AssertionError("MCS %d: %d sites differ, first %s" % (m, len(bad), bad[:4].tolist()))
        mo = lat.measure()
        m_ref = orc.moments(ref)
        for k in ("s1_even", "s1_odd", "s2_even", "s2_odd"):
            assert mo[k] == m_ref[k]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("pq", RATES)
def test_db_rows_every_mcs(okpz, orc, shape, pq):
    D, threads = shape
    _run(okpz, orc, 1024, D, threads, pq[0], pq[1], 3, stream=5)


@pytest.mark.parametrize("shape", SHAPES)
def test_db_rows_longer_run(okpz, orc, shape):
    # a rough surface: many deferred (order-dependent) attempts per round
    D, threads = shape
    _run(okpz, orc, 512, D, threads, 0.95, 0.05, 25, stream=9)
