"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Integer/bit work is compared bit-exactly: the GPU lattice must equal the
oracle's DTr emulation after every MCS.  The moments are exact integers and
the reported doubles (W^2, W^2_sub, C_h) are the exact rationals rounded once,
so they must be equal too.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def lattice(okpz, **kw):
    base = dict(L=64, Dx=16, Dy=16, Cx=8, Cy=8, scheme=0, seed=1, stream=0)
    base.update(kw)
    return okpz.Lattice(base["L"], base["Dx"], base["Dy"], base["Cx"], base["Cy"], base["scheme"],
                        base["seed"], base["stream"], base.get("origin_mode", 0))


def emulator(orc, **kw):
    base = dict(L=64, Dx=16, Dy=16, Cx=8, Cy=8, scheme=0, seed=1, stream=0, p=1.0, q=0.0)
    base.update(kw)
    return orc.Emu(L=base["L"], Dx=base["Dx"], Dy=base["Dy"], Cx=base["Cx"], Cy=base["Cy"],
                   scheme=base["scheme"], p=base["p"], q=base["q"], seed=base["seed"],
                   stream=base["stream"], origin_mode=base.get("origin_mode", 0))


def check_moments(orc, gpu_m, s):
    mo = orc.moments(s)
    for k in ("n_even", "n_odd", "s1_even", "s1_odd", "s2_even", "s2_odd"):
        assert gpu_m[k] == mo[k], k
    assert gpu_m["w2"] == orc.w2_from_moments(mo)
    assert gpu_m["w2_sub"] == orc.w2_sub_from_moments(mo)


def test_philox_device_matches_oracle(okpz, orc):
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 2, 3, 4], [0, 0xFFFFFFFF, 0xFFFFFFFF, 8]]
    for key in ((0, 0), (1, 0), (0xDEADBEEF, 0x12345678)):
        out = okpz.philox(key[0], key[1], ctr)
        for i in range(0, 4096, 7):
            assert tuple(int(v) for v in out[i]) == orc.philox(key, ctr[i])


def test_flat_state_and_moments(okpz, orc):
    for L in (64, 128, 256, 4096):
        with lattice(okpz, L=L, Dx=min(16, L // 2), Dy=min(16, L // 2)) as lat:
            s = lat.sites()
            assert np.array_equal(s, orc.init_flat(L))
            check_moments(orc, lat.measure(), s)


@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_small_config_every_mcs(okpz, orc, scheme):
    # L=64, p=1 q=0, 1000 MCS from flat: bit-exact lattice and exact W^2 after every MCS
    e = emulator(orc, scheme=scheme)
    ref = orc.init_flat(64)
    with lattice(okpz, scheme=scheme) as lat:
        for m in range(1000):
            lat.run(1, 1.0, 0.0)
            e.mcs(ref, m)
            s = lat.sites()
            assert np.array_equal(s, ref), "MCS %d" % m
            if m % 10 == 0 or m < 20:
                check_moments(orc, lat.measure(), ref)


@pytest.mark.parametrize("scheme", [0, 1, 2])
@pytest.mark.parametrize("pq", [(0.95, 0.05), (0.5, 0.5), (0.3, 0.0), (0.0, 0.6), (1.0, 1.0),
                                (0.0, 0.0)])
def test_rates(okpz, orc, scheme, pq):
    p, q = pq
    e = emulator(orc, scheme=scheme, p=p, q=q, stream=3)
    ref = orc.init_flat(64)
    with lattice(okpz, scheme=scheme, stream=3) as lat:
        for m in range(60):
            lat.run(1, p, q)
            e.mcs(ref, m)
            assert np.array_equal(lat.sites(), ref), "MCS %d" % m


SHAPES = [
    # L, Dx, Dy, Cx, Cy : several tiles, cells per domain from 1 to 4096,
    # fewer cells than a wave (ragged workgroups), rectangular domains/cells,
    # domains narrower than a 32-site block (edge blocks shared by two
    # domains of one set) and exactly one block wide
    (64, 16, 16, 2, 2),
    (64, 32, 32, 8, 8),
    (128, 32, 8, 4, 2),
    (128, 8, 32, 2, 8),
    (64, 8, 8, 8, 8),
    (64, 4, 4, 2, 2),
    (128, 32, 16, 4, 2),
    (128, 16, 32, 2, 16),
    (256, 64, 64, 8, 8),
    (256, 128, 64, 4, 4),
    (512, 256, 256, 8, 8),
    (512, 256, 256, 4, 4),
    (512, 128, 128, 2, 2),
    (512, 128, 128, 64, 64),
    (1024, 256, 256, 16, 8),
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_shapes(okpz, orc, shape, scheme):
    L, Dx, Dy, Cx, Cy = shape
    p, q = (0.9, 0.2) if scheme == 1 else (1.0, 0.0)
    e = emulator(orc, L=L, Dx=Dx, Dy=Dy, Cx=Cx, Cy=Cy, scheme=scheme, p=p, q=q, stream=7)
    ref = orc.init_flat(L)
    n = 6 if L <= 256 else 2
    with lattice(okpz, L=L, Dx=Dx, Dy=Dy, Cx=Cx, Cy=Cy, scheme=scheme, stream=7) as lat:
        for m in range(n):
            lat.run(1, p, q)
            e.mcs(ref, m)
            assert np.array_equal(lat.sites(), ref), "MCS %d" % m
        check_moments(orc, lat.measure(), ref)


@pytest.mark.parametrize("mode", [1, 2])
def test_negative_control_origins(okpz, orc, mode):
    e = emulator(orc, scheme=0, origin_mode=mode)
    ref = orc.init_flat(64)
    with lattice(okpz, scheme=0, origin_mode=mode) as lat:
        for m in range(30):
            lat.run(1, 1.0, 0.0)
            e.mcs(ref, m)
        assert np.array_equal(lat.sites(), ref)


@pytest.mark.parametrize("scheme,pq", [(0, (1.0, 0.0)), (1, (0.95, 0.05))])
def test_l4096_full_compare(okpz, orc, scheme, pq):
    # L=4096, 256x256 domains, TC=1,1: whole-lattice bit-exact after each MCS
    p, q = pq
    L = 4096
    e = emulator(orc, L=L, Dx=256, Dy=256, Cx=8, Cy=8, scheme=scheme, p=p, q=q)
    ref = orc.init_flat(L)
    with lattice(okpz, L=L, Dx=256, Dy=256, Cx=8, Cy=8, scheme=scheme) as lat:
        for m in range(2):
            lat.run(1, p, q)
            e.mcs(ref, m)
            assert np.array_equal(lat.sites(), ref), "MCS %d" % m
        check_moments(orc, lat.measure(), ref)
        lat.snapshot()
        s_ref = ref.copy()
        lat.run(1, p, q)
        e.mcs(ref, 2)
        ac = lat.autocorr()
        assert ac["c_h"] == orc.c_h(ref, s_ref)
        assert ac["s_ts"] == orc.cross(ref, s_ref)
        assert ac["overlap"] == orc.slope_overlap(ref, s_ref)
        assert ac["c_s"] == orc.c_s(ref, s_ref)


def test_autocorr_and_snapshot(okpz, orc):
    e = emulator(orc, scheme=1, p=0.95, q=0.05)
    ref = orc.init_flat(64)
    with lattice(okpz, scheme=1) as lat:
        with pytest.raises(okpz.OkpzError):
            lat.autocorr()
        lat.run(5, 0.95, 0.05)
        for m in range(5):
            e.mcs(ref, m)
        lat.snapshot()
        snap = ref.copy()
        ac = lat.autocorr()
        mo = lat.measure()
        assert ac["c_h"] == mo["w2"]  # C_h(s,s) = W^2(s)
        assert ac["c_s"] == 0.25 and ac["overlap"] == 64 * 64  # C_s(s,s) = 1/4
        for m in range(5, 40):
            lat.run(1, 0.95, 0.05)
            e.mcs(ref, m)
            ac = lat.autocorr()
            assert ac["t"] == m + 1 and ac["s"] == 5
            assert ac["s_ts"] == orc.cross(ref, snap)
            assert ac["c_h"] == orc.c_h(ref, snap)
            assert ac["overlap"] == orc.slope_overlap(ref, snap)
            assert ac["c_s"] == orc.c_s(ref, snap)


def test_observe_matches_measure_and_autocorr(okpz, orc):
    e = emulator(orc, L=128, Dx=32, Dy=32, scheme=2, p=0.7, q=0.4)
    ref = orc.init_flat(128)
    with lattice(okpz, L=128, Dx=32, Dy=32, scheme=2) as lat:
        mo, ac = lat.observe(False)
        assert ac is None and mo["w2"] == 0.25
        with pytest.raises(okpz.OkpzError):
            lat.observe(True)
        lat.run(3, 0.7, 0.4)
        for m in range(3):
            e.mcs(ref, m)
        lat.snapshot()
        snap = ref.copy()
        for m in range(3, 9):
            lat.run(1, 0.7, 0.4)
            e.mcs(ref, m)
            mo, ac = lat.observe(True)
            check_moments(orc, mo, ref)
            assert mo == lat.measure()
            assert ac == lat.autocorr()
            assert ac["c_h"] == orc.c_h(ref, snap)
            assert ac["c_s"] == orc.c_s(ref, snap)


@pytest.mark.parametrize("scheme,pq,shape", [(0, (1.0, 0.0), (256, 64, 64, 4, 4)),
                                             (1, (0.95, 0.05), (512, 128, 128, 8, 8)),
                                             (2, (0.7, 0.2), (512, 256, 128, 8, 4))])
def test_workgroup_shape_does_not_change_results(okpz, orc, scheme, pq, shape):
    L, Dx, Dy, Cx, Cy = shape
    e = emulator(orc, L=L, Dx=Dx, Dy=Dy, Cx=Cx, Cy=Cy, scheme=scheme, p=pq[0], q=pq[1])
    ref = orc.init_flat(L)
    for m in range(3):
        e.mcs(ref, m)
    ncell = (Dx // Cx) * (Dy // Cy)
    for threads in (0, 64, 128, 256, 512):
        with lattice(okpz, L=L, Dx=Dx, Dy=Dy, Cx=Cx, Cy=Cy, scheme=scheme) as lat:
            if ncell // threads > 16 if threads else False:
                with pytest.raises(okpz.OkpzError):
                    lat.set_threads(threads)
                continue
            lat.set_threads(threads)
            lat.run(3, *pq)
            assert np.array_equal(lat.sites(), ref), threads


def test_determinism_and_resume(okpz):
    with lattice(okpz, L=256, Dx=64, Dy=64, scheme=1) as a, \
            lattice(okpz, L=256, Dx=64, Dy=64, scheme=1) as b:
        a.run(20, 0.95, 0.05)
        for n in (3, 1, 9, 7):
            b.run(n, 0.95, 0.05)
        assert np.array_equal(a.sites(), b.sites())
        assert a.mcs == b.mcs == 20
        # resume from a host copy with the MCS counter
        s = a.sites()
        a.run(5, 0.95, 0.05)
        b.init_from_host(s, 20)
        b.run(5, 0.95, 0.05)
        assert np.array_equal(a.sites(), b.sites())


def test_init_from_host_roundtrip_and_rejects(okpz, orc):
    sim = orc.SeqRS(64, 0.8, 0.3, seed=2, stream=0)
    sim.run(20)
    with lattice(okpz) as lat:
        lat.init_from_host(sim.s, 0)
        assert np.array_equal(lat.sites(), sim.s)
        assert np.array_equal(lat.heights(), orc.heights(sim.s).astype(np.int32))
        bad = sim.s.copy()
        bad[3, 5] ^= 1
        with pytest.raises(okpz.OkpzError):
            lat.init_from_host(bad, 0)
        bad = sim.s.copy()
        bad[0, 0] |= 4
        with pytest.raises(okpz.OkpzError):
            lat.init_from_host(bad, 0)
        assert np.array_equal(lat.sites(), sim.s)  # unchanged after rejection


def test_window_roundtrip(okpz, orc):
    rng = np.random.default_rng(4)
    with lattice(okpz, L=256, Dx=64, Dy=64) as lat:
        lat.run(3, 1.0, 0.0)
        full = lat.sites()
        for _ in range(20):
            x0, y0 = (int(v) for v in rng.integers(0, 256, 2))
            w, h = (int(v) for v in rng.integers(1, 256, 2))
            win = lat.window(x0, y0, w, h)
            xs, ys = (x0 + np.arange(w)) % 256, (y0 + np.arange(h)) % 256
            assert np.array_equal(win, full[np.ix_(ys, xs)])
        # write back a modified window and read it again
        piece = full[10:30, 250 - 256:].copy() if False else full[np.ix_(np.arange(10, 30),
                                                                         (250 + np.arange(12)) % 256)]
        lat.set_window(250, 10, piece)
        assert np.array_equal(lat.sites(), full)


def test_external_torch_buffer(okpz, orc):
    torch = pytest.importorskip("torch")
    L = 128
    buf = torch.zeros(L * L // 16, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    lat = okpz.Lattice(L, 32, 32, 8, 8, 1, 1, 0, 0, hip_stream=stream,
                       device_buffer=(buf.data_ptr(), buf.numel() * 4))
    e = emulator(orc, L=L, Dx=32, Dy=32, scheme=1, p=0.95, q=0.05)
    ref = orc.init_flat(L)
    lat.run(4, 0.95, 0.05)
    for m in range(4):
        e.mcs(ref, m)
    torch.cuda.synchronize()
    words = buf.cpu().numpy().view(np.uint32)
    assert np.array_equal(words, lat.words())
    assert np.array_equal(lat.sites(), ref)
    lat.close()


def test_bad_arguments(okpz):
    with lattice(okpz) as lat:
        with pytest.raises(okpz.OkpzError):
            lat.run(1, 1.5, 0.0)
        with pytest.raises(okpz.OkpzError):
            lat.run(1, 0.5, -0.1)
        with pytest.raises(okpz.OkpzError):
            lat.window(0, 0, 0, 4)
        with pytest.raises(okpz.OkpzError):
            okpz.Lattice(96, 16, 16, 8, 8)
