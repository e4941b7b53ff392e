"""Parity of the dead-border device layer (the cDB negative control with the
coarse origin, Sec. 4.1) with the oracle's emulation, bit for bit after every
MCS: all tiles of one launch border each other, so the words they share go
back as XORs of the change, and attempts on a tile's last column or row are
not carried out.  Every block scheme, every origin mode, domains narrower than
a word, one word, several words and the 256-site shape the specialised
kernels would otherwise take."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (L, D, C, threads)
SHAPES = [(128, 16, 8, 0), (256, 32, 8, 0), (256, 64, 8, 64), (512, 256, 8, 0)]
ORIGINS = ["random", "fixed", "coarse"]


def _run(okpz, orc, L, D, C, threads, scheme, origin, p, q, n_mcs, stream):
    sch = {"DT": (orc.DT, okpz.BLOCK_DT), "DB": (orc.DB, okpz.BLOCK_DB), "DTr": (orc.DTR, okpz.BLOCK_DTR)}[scheme]
    om = {"random": (orc.ORIGIN_RANDOM, okpz.ORIGIN_RANDOM), "fixed": (orc.ORIGIN_FIXED, okpz.ORIGIN_FIXED),
          "coarse": (orc.ORIGIN_COARSE, okpz.ORIGIN_COARSE)}[origin]
    e = orc.Emu(L=L, Dx=D, Dy=D, Cx=C, Cy=C, scheme=sch[0], p=p, q=q, seed=17, stream=stream,
                origin_mode=om[0], device=orc.DEVICE_DB)
    ref = orc.init_flat(L)
    with okpz.Lattice(L, D, D, C, C, sch[1], 17, stream, origin_mode=om[1], device_layer=okpz.DEVICE_DB) as lat:
        if threads:
            lat.set_threads(threads)
        for m in range(n_mcs):
            print("dead border: L=%d D=%d threads=%d %s %s p=%r q=%r MCS %d" % (L, D, threads, scheme, origin, p, q, m),
                  flush=True)
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
@pytest.mark.parametrize("scheme", ["DT", "DB", "DTr"])
@pytest.mark.parametrize("origin", ORIGINS)
def test_dead_border_every_mcs(okpz, orc, shape, scheme, origin):
    L, D, C, threads = shape
    _run(okpz, orc, L, D, C, threads, scheme, origin, 0.95, 0.05, 3, stream=3)


@pytest.mark.parametrize("pq", [(1.0, 0.0), (0.5, 0.5), (0.0, 1.0)])
@pytest.mark.parametrize("scheme", ["DT", "DB", "DTr"])
def test_dead_border_rates(okpz, orc, pq, scheme):
    _run(okpz, orc, 256, 32, 8, 0, scheme, "coarse", pq[0], pq[1], 4, stream=4)


def test_dead_border_longer_run(okpz, orc):
    # a rough surface at the cDB control's shape (coarse origin, block DB)
    _run(okpz, orc, 256, 64, 8, 0, "DB", "coarse", 0.95, 0.05, 30, stream=8)


def test_dead_border_rejected_by_batches(okpz):
    b = okpz.Batch()
    with okpz.Lattice(256, 32, 32, 8, 8, okpz.BLOCK_DT, 1, 0, hip_stream=b.hip_stream,
                      device_layer=okpz.DEVICE_DB) as lat:
        with pytest.raises(okpz.OkpzError) as err:
            b.add(lat)
        assert err.value.status == okpz.EINVAL
    with okpz.Lattice(256, 32, 32, 8, 8, okpz.BLOCK_DT, 1, 0, hip_stream=b.hip_stream) as lat:
        b.add(lat)  # the same lattice with double tiling joins
        b.remove(lat.slot)
    b.close()


def _slope_ac(okpz, L, D, origin, n, s, ratios):
    """Mean and SE of C_s(t, s) over n single lattices (streams 0 .. n-1) of
    the dead-border layer with block DT at p = 1, at t = s * ratio."""
    lats = [okpz.Lattice(L, D, D, 8, 8, okpz.BLOCK_DT, 3, r, origin_mode=origin, device_layer=okpz.DEVICE_DB)
            for r in range(n)]
    try:
        for lat in lats:
            lat.run(s, 1.0, 0.0)
            lat.snapshot()
        out, t = [], s
        for rr in ratios:
            for lat in lats:
                lat.run(s * rr - t, 1.0, 0.0)
            t = s * rr
            cs = np.array([lat.observe(True)[1]["c_s"] for lat in lats])
            out.append((cs.mean(), cs.std(ddof=1) / np.sqrt(n)))
            print("dead border origin=%d L=%d t/s=%d C_s=%.3e +- %.1e" % (origin, L, rr, *out[-1]), flush=True)
        return out
    finally:
        for lat in lats:
            lat.close()


def test_coarse_dead_border_imprints_a_slope_pattern(okpz):
    """The paper's cDB artifact (Sec. 4.1): with the origin on the 4x4 grid
    only sites with x or y = 3 (mod 4) are ever dead, and the slope
    autocorrelation stops decaying at a finite value; a freely moving origin
    removes it.  L = 4096, D = 64, 128 lattices per origin, s = 100 MCS."""
    L, D, n, s = 4096, 64, 128, 100
    cdb = _slope_ac(okpz, L, D, okpz.ORIGIN_COARSE, n, s, [10, 20])
    dbr = _slope_ac(okpz, L, D, okpz.ORIGIN_RANDOM, n, s, [10, 20])
    for (mc, ec), (mr, er) in zip(cdb, dbr):
        assert mc - mr > 4.0 * np.hypot(ec, er), (mc, ec, mr, er)
    # no decay between t/s = 10 and 20 (the random origin's C_s falls several-fold there)
    assert cdb[1][0] > 0.6 * cdb[0][0]
