"""The oracle's dead-border device layer (Sec. 3 DB; with the coarse origin the
cDB of Sec. 4.1): every tile of Dx x Dy sites is swept in one step per MCS
and the sites of its last column and last row are inactive.  Pinned against
what the scheme fixes, independently of the emulation's own bookkeeping:

* an inactive site is never updated, so the height difference between any
  two inactive sites (absolute heights change only where a site is updated)
  is the same after every MCS when the origin is fixed;
* the hit counts are zero on the dead rims, and L^2 attempts are drawn per
  MCS;
* the tiles do not interact, so sweeping them in reverse or shuffled order
  gives the same lattice bit for bit;
* the update rule keeps the state a height configuration.
"""
import numpy as np
import pytest

import oracle as orc

pytestmark = pytest.mark.filterwarnings("ignore")


def _emu(L, D, scheme, p, q, origin, **kw):
    return orc.Emu(L=L, Dx=D, Dy=D, Cx=min(8, D), Cy=min(8, D), scheme=scheme, p=p, q=q, seed=5, stream=2,
                   origin_mode=origin, device=orc.DEVICE_DB, **kw)


def _rim_mask(L, D):
    x = np.arange(L)
    col = (x % D) == D - 1
    return col[None, :] | col[:, None]


@pytest.mark.parametrize("scheme", [orc.DT, orc.DB, orc.DTR], ids=["DT", "DB", "DTr"])
@pytest.mark.parametrize("pq", [(1.0, 0.0), (0.6, 0.4)])
def test_dead_sites_never_move(scheme, pq):
    L, D = 64, 16
    e = _emu(L, D, scheme, pq[0], pq[1], orc.ORIGIN_FIXED)
    s = orc.init_flat(L)
    rim = _rim_mask(L, D)
    ref_site = tuple(np.argwhere(rim)[0])
    h = orc.heights(s)
    before = h[rim] - h[ref_site]
    moved = 0
    for m in range(12):
        e.mcs(s, m)
        assert orc.check_state(s) == 0
        h = orc.heights(s)
        assert np.array_equal(h[rim] - h[ref_site], before), m
        moved += int(np.count_nonzero(h[~rim] - h[ref_site] != 0))
    assert moved > 0  # the active sites do move


@pytest.mark.parametrize("origin", [orc.ORIGIN_FIXED, orc.ORIGIN_COARSE, orc.ORIGIN_RANDOM])
def test_hits_avoid_the_rim(origin):
    L, D = 64, 16
    e = _emu(L, D, orc.DB, 0.95, 0.05, origin)
    s = orc.init_flat(L)
    for m in range(6):
        hits = np.zeros((L, L), dtype=np.uint32)
        assert e.mcs(s, m, hits) == L * L  # drawn attempts, void ones included
        ox, oy, _ = e.mcs_draw(m)
        if origin == orc.ORIGIN_COARSE:
            assert ox % 4 == 0 and oy % 4 == 0
        rim = np.roll(np.roll(_rim_mask(L, D), ox, axis=1), oy, axis=0)
        assert hits[rim].sum() == 0
        # the void share is the rim's share of the sites, about 2/D
        assert 0.75 * (2 * D - 1) / D ** 2 < 1 - hits.sum() / (L * L) < 1.25 * (2 * D - 1) / D ** 2


@pytest.mark.parametrize("scheme", [orc.DT, orc.DB, orc.DTR], ids=["DT", "DB", "DTr"])
def test_tile_order_does_not_matter(scheme):
    L, D = 64, 16
    ref = orc.init_flat(L)
    e0 = _emu(L, D, scheme, 0.8, 0.3, orc.ORIGIN_COARSE)
    for m in range(5):
        e0.mcs(ref, m)
    for order in (1, 2):
        s = orc.init_flat(L)
        e = _emu(L, D, scheme, 0.8, 0.3, orc.ORIGIN_COARSE, order=order, order_seed=77)
        for m in range(5):
            e.mcs(s, m)
        assert np.array_equal(s, ref), order


def test_validation():
    assert _emu(64, 64, orc.DB, 1.0, 0.0, orc.ORIGIN_COARSE).validate()  # one tile spanning the lattice
    assert not _emu(64, 128, orc.DB, 1.0, 0.0, orc.ORIGIN_COARSE).validate()
    e = orc.Emu(L=64, Dx=64, Dy=64, Cx=8, Cy=8, scheme=orc.DB, p=1.0, q=0.0)  # double tiling needs 2D <= L
    assert not e.validate()
