"""Parity of the row-paired DT / DTr device step (square 128- and 256-site
domains, 8 x 8-site cells, one to four cells per lane) with the oracle's DTr
emulation, bit for bit after every MCS: every workgroup shape that selects
it, both block schemes, rates with and without acceptance prefixes, rates
whose thresholds tie often (the 32-bit tie-break draw decides), and both
stochastic directions."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (Dx, threads): 256-site domains have 1024 cells (512 lanes: 2 per lane,
# 256 lanes: 4); 128-site domains have 256 cells (256 lanes: 1, 128: 2, 64: 4)
SHAPES = [(256, 512), (256, 256), (128, 256), (128, 128), (128, 64)]
RATES = [(1.0, 0.0), (0.95, 0.05), (0.5, 0.5), (0.3, 0.9), (0.0, 1.0), (1.0, 1.0),
         # 12-bit prefixes: P = 4095/4096 + 2^-22 ties at prefix 4095 with a nonzero low word
         (4095 / 4096 + 2.0 ** -22, 1 / 4096 + 2.0 ** -23)]


def _run(okpz, orc, L, D, threads, scheme, p, q, n_mcs, stream):
    sch = {"DT": (orc.DT, okpz.BLOCK_DT), "DTr": (orc.DTR, okpz.BLOCK_DTR)}[scheme]
    e = orc.Emu(L=L, Dx=D, Dy=D, Cx=8, Cy=8, scheme=sch[0], p=p, q=q, seed=13, stream=stream)
    ref = orc.init_flat(L)
    with okpz.Lattice(L, D, D, 8, 8, sch[1], 13, stream) as lat:
        lat.set_threads(threads)
        for m in range(n_mcs):
            print("dt_rows: L=%d D=%d threads=%d %s p=%r q=%r MCS %d" % (L, D, threads, scheme, p, q, m), flush=True)
            lat.run(1, p, q)
            e.mcs(ref, m)
            got = lat.sites()
            if not np.array_equal(got, ref):
                bad = np.argwhere(got != ref)
                raise AssertionError("MCS %d: %d sites differ, first %s" % (m, len(bad), bad[:4].tolist()))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("scheme", ["DT", "DTr"])
@pytest.mark.parametrize("pq", RATES)
def test_dt_rows_every_mcs(okpz, orc, shape, scheme, pq):
    D, threads = shape
    _run(okpz, orc, 1024, D, threads, scheme, pq[0], pq[1], 3, stream=6)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("scheme", ["DT", "DTr"])
def test_dt_rows_longer_run(okpz, orc, shape, scheme):
    D, threads = shape
    _run(okpz, orc, 512, D, threads, scheme, 0.95, 0.05, 25, stream=10)
