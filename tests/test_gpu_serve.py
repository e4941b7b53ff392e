"""Serving with continuous batching: every request's result equals the same
simulation run alone, bit for bit, whatever else shares the GPU with it and
whenever it arrived; admission respects the HBM budget and member limit."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (L, D, C, n_mcs, p): DB (the serving scheme), q = 1 - p
REQUESTS = [
    (64, 16, 8, 5, 0.9),
    (128, 32, 8, 7, 0.6),
    (256, 128, 8, 4, 0.75),
    (64, 8, 4, 9, 1.0),
    (128, 64, 8, 2, 0.5),
    (256, 64, 8, 6, 0.95),
    (64, 32, 8, 3, 0.7),
    (128, 16, 8, 8, 0.55),
    (64, 16, 8, 1, 0.8),
    (256, 32, 4, 5, 0.65),
]


def alone(okpz, L, D, C, n, p, stream, scheme=None):
    scheme = okpz.BLOCK_DB if scheme is None else scheme
    with okpz.Lattice(L, D, D, C, C, scheme, seed=3, stream=stream) as lat:
        lat.run(n, p, 1.0 - p)
        return lat.sites(), lat.measure()


def test_served_results_equal_alone(okpz, orc):
    srv = okpz.Server(chunk_mcs=3, max_members=4)
    ids = {}
    for k, (L, D, C, n, p) in enumerate(REQUESTS):
        rid = srv.submit(L, D, D, C, C, okpz.BLOCK_DB, 3, 500 + k, n, p, 1.0 - p, want_sites=True)
        ids[rid] = k
        if k % 3 == 2:
            time.sleep(0.02)  # later requests arrive while earlier ones run
    srv.drain(120.0)
    res = srv.poll()
    st = srv.stats()
    srv.close()
    assert len(res) == len(REQUESTS) and st["finished"] == st["submitted"] == len(REQUESTS)
    assert 1 <= st["max_members"] <= 4
    for r in res:
        k = ids[r["id"]]
        L, D, C, n, p = REQUESTS[k]
        assert r["status"] == 0 and r["L"] == L and r["n_mcs"] == n
        assert r["t_submit"] <= r["t_start"] <= r["t_finish"]
        sites, mo = alone(okpz, L, D, C, n, p, 500 + k)
        assert np.array_equal(r["sites"], sites), k
        assert r["moments"] == mo
        if L == 64:
            emu = orc.Emu(L=L, Dx=D, Dy=D, Cx=C, Cy=C, scheme=orc.DB, p=p, q=1.0 - p, seed=3, stream=500 + k)
            ref = orc.init_flat(L)
            for m in range(n):
                emu.mcs(ref, m)
            assert np.array_equal(r["sites"], ref), k
            assert r["moments"]["w2"] == orc.w2(ref)


def test_admission_respects_budget(okpz):
    # room for exactly one L=256 lattice: requests then run one at a time
    one = 256 * 256 // 4 + 256 * 4 + 64 * 6 * 8 + 12 * 8
    srv = okpz.Server(hbm_budget=one + 100, chunk_mcs=2)
    for k in range(4):
        srv.submit(256, 64, 64, 8, 8, okpz.BLOCK_DB, 3, 700 + k, 3, 0.8, 0.2)
    with pytest.raises(okpz.OkpzError):
        srv.submit(512, 64, 64, 8, 8, okpz.BLOCK_DB, 3, 9, 3, 0.8, 0.2)  # can never fit
    srv.drain(120.0)
    res = srv.poll()
    st = srv.stats()
    srv.close()
    assert len(res) == 4 and st["max_members"] == 1
    res.sort(key=lambda r: r["id"])
    for a, b in zip(res, res[1:]):  # FIFO, one after the other
        assert a["t_finish"] <= b["t_start"]


def test_server_rejects_bad_requests(okpz):
    srv = okpz.Server()
    with pytest.raises(okpz.OkpzError):
        srv.submit(64, 16, 16, 8, 8, okpz.BLOCK_DB, 1, 0, 0, 0.5, 0.5)     # no MCS
    with pytest.raises(okpz.OkpzError):
        srv.submit(64, 16, 16, 8, 8, okpz.BLOCK_DB, 1, 0, 5, 1.5, 0.0)     # p > 1
    with pytest.raises(okpz.OkpzError):
        srv.submit(96, 16, 16, 8, 8, okpz.BLOCK_DB, 1, 0, 5, 0.5, 0.5)     # L not a power of 2
    srv.drain(10.0)
    assert srv.poll() == []
    srv.close()


def test_mixed_block_schemes_equal_alone(okpz, orc):
    """Requests of different block schemes arriving interleaved are served
    together (one batch per scheme in every tick) and each equals its run alone."""
    schemes = [okpz.BLOCK_DT, okpz.BLOCK_DB, okpz.BLOCK_DTR]
    orc_scheme = {okpz.BLOCK_DT: orc.DT, okpz.BLOCK_DB: orc.DB, okpz.BLOCK_DTR: orc.DTR}
    reqs = [(64, 16, 8, 5, 0.9), (128, 32, 8, 4, 0.6), (64, 32, 8, 6, 1.0), (256, 64, 8, 3, 0.75),
            (64, 16, 4, 7, 0.55), (128, 64, 8, 5, 0.95)]
    srv = okpz.Server(chunk_mcs=2, max_members=8)
    ids = {}
    for k, (L, D, C, n, p) in enumerate(reqs):
        sch = schemes[k % 3]
        rid = srv.submit(L, D, D, C, C, sch, 3, 800 + k, n, p, 1.0 - p, want_sites=True)
        ids[rid] = (k, sch)
    srv.drain(120.0)
    res = srv.poll()
    st = srv.stats()
    srv.close()
    assert len(res) == len(reqs) and st["finished"] == len(reqs)
    assert st["max_members"] >= 2  # schemes were resident together
    for r in res:
        k, sch = ids[r["id"]]
        L, D, C, n, p = reqs[k]
        assert r["status"] == 0, (k, sch, r["status"])
        sites, mo = alone(okpz, L, D, C, n, p, 800 + k, sch)
        assert np.array_equal(r["sites"], sites), (k, sch)
        assert r["moments"] == mo
        if L == 64:
            emu = orc.Emu(L=L, Dx=D, Dy=D, Cx=C, Cy=C, scheme=orc_scheme[sch], p=p, q=1.0 - p, seed=3,
                          stream=800 + k)
            ref = orc.init_flat(L)
            for m in range(n):
                emu.mcs(ref, m)
            assert np.array_equal(r["sites"], ref), (k, sch)


def test_served_serving_size_equals_alone(okpz):
    """A request at serving size (L = 2048, D = 256, the column sweep of the
    serving workload) beside small ones equals its run alone."""
    reqs = [(2048, 256, 8, 6, 0.8), (256, 64, 8, 9, 0.7), (512, 256, 8, 4, 0.95)]
    srv = okpz.Server(chunk_mcs=2, max_members=4)
    ids = {}
    for k, (L, D, C, n, p) in enumerate(reqs):
        ids[srv.submit(L, D, D, C, C, okpz.BLOCK_DB, 3, 900 + k, n, p, 1.0 - p, want_sites=True)] = k
    srv.drain(300.0)
    res = srv.poll()
    srv.close()
    assert len(res) == len(reqs)
    for r in res:
        k = ids[r["id"]]
        L, D, C, n, p = reqs[k]
        assert r["status"] == 0
        sites, mo = alone(okpz, L, D, C, n, p, 900 + k)
        assert np.array_equal(r["sites"], sites), k
        assert r["moments"] == mo
