"""Checkpoint and resume: a run interrupted by okpz_save / okpz_load into a
fresh lattice continues bit-identically to the uninterrupted run (random
draws depend only on the parameters and the MCS index), the restored state
is the oracle's DTr emulation at that MCS, and damaged or foreign blobs are
rejected without touching the lattice."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HEADER = 128
P, Q = 0.95, 0.05


def ckp_checksum(blob: np.ndarray) -> int:
    """The blob's checksum: multiply-xor over 8-byte units of the header (its
    checksum field zeroed) and then the payload."""
    head = blob[:HEADER].copy()
    head[80:88] = 0  # checksum field: after magic 8, version 4, flags 4, params 40, 3 x uint64
    h = 0xCBF29CE484222325
    m = (1 << 64) - 1
    for part in (head, blob[HEADER:]):
        for v in part.view(np.uint64).tolist():
            h = ((h ^ v) * 0x100000001B3) & m
            h ^= h >> 29
    return h


@pytest.mark.parametrize("scheme", [0, 1, 2], ids=["DT", "DB", "DTr"])
def test_resume_is_bit_identical(okpz, orc, scheme):
    L, D, C = 128, 32, 8
    a = okpz.Lattice(L, D, D, C, C, scheme, seed=21, stream=4)
    a.run(3, P, Q)
    a.snapshot()
    a.run(2, P, Q)
    blob = a.save(with_snapshot=True)
    assert blob.size == HEADER + 2 * L * L // 4
    at_save = a.sites()
    # the saved state is the oracle's emulation at MCS 5
    emu = orc.Emu(L=L, Dx=D, Dy=D, Cx=C, Cy=C, scheme=scheme, p=P, q=Q, seed=21, stream=4)
    s = orc.init_flat(L)
    for m in range(5):
        emu.mcs(s, m)
    assert np.array_equal(at_save, s)
    a.run(4, P, Q)
    ref_sites = a.sites()
    ref_obs = a.observe(with_autocorr=True)

    b = okpz.Lattice(L, D, D, C, C, scheme, seed=21, stream=4)
    b.run(1, 1.0, 0.0)  # some other state, overwritten by the load
    b.load(blob)
    assert b.mcs == 5
    assert np.array_equal(b.sites(), at_save)
    b.run(4, P, Q)
    assert np.array_equal(b.sites(), ref_sites)
    assert b.observe(with_autocorr=True) == ref_obs
    a.close()
    b.close()


def test_checkpoint_without_snapshot(okpz):
    a = okpz.Lattice(64, 16, 16, 8, 8, 1, seed=2, stream=0)
    with pytest.raises(okpz.OkpzError) as e:
        a.save(with_snapshot=True)
    assert e.value.status == okpz.ESTATE
    a.run(2, P, Q)
    blob = a.save()
    assert blob.size == HEADER + 64 * 64 // 4
    b = okpz.Lattice(64, 16, 16, 8, 8, 1, seed=2, stream=0)
    b.snapshot()
    b.load(blob)  # a blob without a snapshot clears the lattice's snapshot
    with pytest.raises(okpz.OkpzError) as e:
        b.autocorr()
    assert e.value.status == okpz.ESTATE
    assert b.measure() == a.measure()
    a.close()
    b.close()


def test_load_rejects_bad_blobs(okpz):
    L = 64
    a = okpz.Lattice(L, 16, 16, 8, 8, 1, seed=5, stream=1)
    a.run(3, P, Q)
    blob = a.save()
    assert ckp_checksum(blob) == int(blob[80:88].view(np.uint64)[0])
    b = okpz.Lattice(L, 16, 16, 8, 8, 1, seed=5, stream=1)
    b.run(1, P, Q)
    before = b.sites()

    def rejected(bad):
        with pytest.raises(okpz.OkpzError) as e:
            b.load(bad)
        assert e.value.status == okpz.EINVAL
        assert np.array_equal(b.sites(), before) and b.mcs == 1

    rejected(blob[:-8])  # short
    bad = blob.copy()
    bad[0] ^= 1  # magic
    rejected(bad)
    bad = blob.copy()
    bad[HEADER + 100] ^= 4  # payload bit: checksum mismatch
    rejected(bad)
    # a state that is not a height configuration, with a correct checksum:
    # sx(0, 0) flipped leaves the plaquettes at (0, 0) and (0, 1) open
    bad = blob.copy()
    bad[HEADER] ^= 1
    bad[80:88] = np.array([ckp_checksum(bad)], dtype=np.uint64).view(np.uint8)
    rejected(bad)
    other = okpz.Lattice(L, 16, 16, 8, 8, 1, seed=6, stream=1)  # another seed
    with pytest.raises(okpz.OkpzError) as e:
        other.load(blob)
    assert e.value.status == okpz.EINVAL
    b.load(blob)
    assert np.array_equal(b.sites(), a.sites()) and b.mcs == 3
    for lat in (a, b, other):
        lat.close()
