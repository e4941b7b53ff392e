"""The allocation-free measurement entry point gives exactly what
okpz_measure gives on the same lattice: two calls in a row, the second on a
smaller lattice, each against the handle-based call (integers equal, doubles
equal), plus the asynchronous form read back from the caller's buffer."""
import pytest

pytestmark = pytest.mark.gpu


def _check_against_measure(okpz, torch, totals, L, D, scheme, n_mcs, p, q, seed):
    with okpz.Lattice(L, D, D, 8, 8, scheme, seed=seed, stream=L) as lat:
        lat.run(n_mcs, p, q)
        ref = lat.measure()
        ptr, nbytes = lat.device_words()
        assert nbytes == L * L // 4
        print("noalloc: L=%d D=%d scheme=%d mcs=%d seed=%d" % (L, D, scheme, n_mcs, seed), flush=True)
        got = okpz.measure_noalloc(ptr, L, totals.data_ptr())
        for k in ("n_even", "n_odd", "s1_even", "s1_odd", "s2_even", "s2_odd", "w2", "w2_sub"):
            assert got[k] == ref[k], (k, got[k], ref[k])
        assert got["mcs"] == 0
        # the totals the call left in the caller's buffer: four exact int128
        # sums as (lo, hi) pairs, then two zero pairs
        t = totals.cpu().tolist()
        as_i128 = [((t[2 * i + 1] << 64) | (t[2 * i] & (2 ** 64 - 1))) for i in range(6)]
        assert as_i128 == [ref["s1_even"], ref["s1_odd"], ref["s2_even"], ref["s2_odd"], 0, 0]
        # asynchronous form: only the kernels are queued; the buffer holds the totals afterwards
        totals.fill_(-7)
        torch.cuda.synchronize()
        assert okpz.measure_noalloc(ptr, L, totals.data_ptr(), synchronous=False) is None
        torch.cuda.synchronize()
        assert totals.cpu().tolist() == t
        return got


def test_noalloc_equals_measure_twice_second_smaller(okpz):
    import torch

    totals = torch.zeros(12, dtype=torch.int64, device="cuda")
    a = _check_against_measure(okpz, torch, totals, 1024, 128, okpz.BLOCK_DB, 9, 0.95, 0.05, seed=5)
    b = _check_against_measure(okpz, torch, totals, 256, 32, okpz.BLOCK_DT, 6, 1.0, 0.0, seed=6)
    assert a["w2"] != b["w2"]


def test_noalloc_largest_lattice_and_flat(okpz):
    # the scratch array's limit: L = 2^17 (flat state, closed form W^2 = 1/4)
    import torch

    totals = torch.zeros(12, dtype=torch.int64, device="cuda")
    L = 1 << 17
    with okpz.Lattice(L, 256, 256, 8, 8, okpz.BLOCK_DB, seed=1, stream=0) as lat:
        ptr, _ = lat.device_words()
        print("noalloc: flat L=2^17", flush=True)
        got = okpz.measure_noalloc(ptr, L, totals.data_ptr())
        assert got["w2"] == 0.25 and got["w2_sub"] == 0.0
        ref = lat.measure()
        for k in ("s1_even", "s1_odd", "s2_even", "s2_odd"):
            assert got[k] == ref[k]
