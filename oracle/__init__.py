"""CPU oracle for the octahedron model with DTr domain decomposition.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It wraps the plain C
implementation in ``octa_oracle.c`` (built with gcc, no GPU code, no code shared
with the HIP library) and adds exact-rational post-processing in Python.

Paper: Kelling, Odor, Gemming, arXiv:1705.01022.
  * update rule ............ Sec. 2.1 (Kawasaki dimer exchange)
  * W^2, C_h ............... Sec. 2.1 (roughness definition, height autocorrelation)
  * sequential RS .......... Sec. 1, Sec. 4.3 (the CPU reference)
  * DTr, DT, DB ............ Sec. 3 and Sec. 3.1 (device and block layer)

State arrays are numpy ``uint8`` of shape ``(L, L)`` indexed ``[y, x]``:
bit 0 = sx (slope to the left neighbour is +1), bit 1 = sy (slope to the
neighbour above, i.e. at y-1, is +1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "octa_oracle.c")
_LIB = os.path.join(_HERE, "liboctaoracle.so")

DT, DB, DTR = 0, 1, 2
SCHEMES = {"DT": DT, "DB": DB, "DTR": DTR, "DTr": DTR}
ORIGIN_RANDOM, ORIGIN_FIXED, ORIGIN_COARSE = 0, 1, 2
# device layer: double tiling (four domain sets per MCS) or dead border (every
# tile at once, its last column and row inactive; Sec. 3 DB, cDB with ORIGIN_COARSE)
DEVICE_DT, DEVICE_DB = 0, 1


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc into ``oracle/liboctaoracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class DtrCfg(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_uint32),
        ("Dx", ctypes.c_uint32),
        ("Dy", ctypes.c_uint32),
        ("Cx", ctypes.c_uint32),
        ("Cy", ctypes.c_uint32),
        ("scheme", ctypes.c_int32),
        ("seed", ctypes.c_uint32),
        ("stream", ctypes.c_uint32),
        ("p", ctypes.c_double),
        ("q", ctypes.c_double),
        ("wx0", ctypes.c_uint32),
        ("wy0", ctypes.c_uint32),
        ("W", ctypes.c_uint32),
        ("H", ctypes.c_uint32),
        ("order", ctypes.c_int32),
        ("order_seed", ctypes.c_uint64),
        ("check_adjacency", ctypes.c_int32),
        ("origin_mode", ctypes.c_int32),
        ("device", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        _lib.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        _lib.orc_init_flat.argtypes = [u8p, ctypes.c_uint32]
        _lib.orc_check_state.argtypes = [u8p, ctypes.c_uint32]
        _lib.orc_check_state.restype = ctypes.c_int
        _lib.orc_attempt.argtypes = [u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_int, ctypes.c_int]
        _lib.orc_attempt.restype = ctypes.c_int
        _lib.orc_seq_init.argtypes = [u64p, ctypes.c_uint64, ctypes.c_uint64]
        _lib.orc_seq_mcs.argtypes = [u8p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                     ctypes.c_double, u64p]
        _lib.orc_seq_mcs.restype = ctypes.c_int64
        _lib.orc_dtr_validate.argtypes = [ctypes.POINTER(DtrCfg)]
        _lib.orc_dtr_validate.restype = ctypes.c_int
        _lib.orc_mcs_draw.argtypes = [ctypes.POINTER(DtrCfg), ctypes.c_uint32, u32p]
        _lib.orc_dtr_mcs.argtypes = [u8p, u8p, ctypes.POINTER(DtrCfg), ctypes.c_uint32,
                                     ctypes.POINTER(ctypes.c_int32), u32p]
        _lib.orc_dtr_mcs.restype = ctypes.c_int64
        _lib.orc_heights.argtypes = [u8p, ctypes.c_uint32, i64p]
        _lib.orc_moments.argtypes = [u8p, ctypes.c_uint32, i64p]
        _lib.orc_moments.restype = ctypes.c_int
        _lib.orc_cross.argtypes = [u8p, u8p, ctypes.c_uint32, i64p]
        _lib.orc_cross.restype = ctypes.c_int
        _lib.orc_slope_overlap.argtypes = [u8p, u8p, ctypes.c_uint32]
        _lib.orc_slope_overlap.restype = ctypes.c_int64
        _lib.orc_cfg_size.restype = ctypes.c_uint32
        if _lib.orc_cfg_size() != ctypes.sizeof(DtrCfg):
            raise RuntimeError("oracle config struct layout mismatch")
    return _lib


def _u8(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _i64(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _u32(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


# --------------------------------------------------------------------------- Philox
def philox(key, ctr) -> tuple:
    """Philox4x32-10 block for key (k0, k1) and counter (c0, c1, c2, c3)."""
    k = np.asarray(key, dtype=np.uint32)
    c = np.asarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_u32(k), _u32(c), _u32(out))
    return tuple(int(v) for v in out)


# --------------------------------------------------------------------------- state
def init_flat(L: int) -> np.ndarray:
    s = np.zeros((L, L), dtype=np.uint8)
    lib().orc_init_flat(_u8(s), L)
    return s


def check_state(s: np.ndarray) -> int:
    return lib().orc_check_state(_u8(s), s.shape[0])


def attempt(s: np.ndarray, x: int, y: int, dep_ok: bool, rem_ok: bool) -> int:
    return lib().orc_attempt(_u8(s), s.shape[0], x, y, int(dep_ok), int(rem_ok))


# --------------------------------------------------------------------------- sequential RS
class SeqRS:
    """Sequential random-sequential dynamics with its own xoshiro256** stream."""

    def __init__(self, L: int, p: float, q: float, seed: int = 1, stream: int = 0):
        self.L, self.p, self.q = L, p, q
        self.state = np.zeros(4, dtype=np.uint64)
        lib().orc_seq_init(self.state.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), seed, stream)
        self.s = init_flat(L)
        self.mcs = 0

    def run(self, n_mcs: int) -> int:
        net = lib().orc_seq_mcs(_u8(self.s), self.L, n_mcs, self.p, self.q,
                                self.state.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
        self.mcs += n_mcs
        return net


def _seq_roughness_rows(args) -> list:
    L, p, q, times, seed, streams = args
    rows = []
    for r in streams:
        rs = SeqRS(L, p, q, seed=seed, stream=r)
        t, row = 0, []
        for tt in times:
            rs.run(tt - t)
            t = tt
            row.append(w2(rs.s))
        rows.append(row)
    return rows


def seq_rs_roughness(L: int, p: float, q: float, times, seed: int, n: int, workers: int = 1) -> np.ndarray:
    """W^2 at each of ``times`` (MCS, non-decreasing) of n sequential-RS runs
    from the flat state (streams 0 .. n-1 of ``seed``): rows are runs.  With
    workers > 1 the runs are spread over freshly spawned processes (the rows
    do not depend on how)."""
    times = list(times)
    if workers <= 1:
        return np.array(_seq_roughness_rows((L, p, q, times, seed, list(range(n)))))
    import multiprocessing as mp

    chunks = [list(range(k, n, workers)) for k in range(workers)]
    with mp.get_context("spawn").Pool(workers) as pool:
        parts = pool.map(_seq_roughness_rows, [(L, p, q, times, seed, c) for c in chunks])
    out = np.zeros((n, len(times)))
    for c, rows in zip(chunks, parts):
        for r, row in zip(c, rows):
            out[r] = row
    return out


# --------------------------------------------------------------------------- DTr emulation
@dataclass
class Emu:
    """Parameters of the DTr emulation (device DTr + block DT/DB/DTr; device
    dead border with ``device=DEVICE_DB``)."""

    L: int
    Dx: int
    Dy: int
    Cx: int
    Cy: int
    scheme: int
    p: float
    q: float
    seed: int = 1
    stream: int = 0
    order: int = 0
    order_seed: int = 0
    check_adjacency: bool = False
    origin_mode: int = ORIGIN_RANDOM
    device: int = DEVICE_DT

    def cfg(self, window=None) -> DtrCfg:
        wx0, wy0, W, H = window if window is not None else (0, 0, self.L, self.L)
        return DtrCfg(self.L, self.Dx, self.Dy, self.Cx, self.Cy, self.scheme, self.seed,
                      self.stream, float(self.p), float(self.q), wx0, wy0, W, H, self.order,
                      self.order_seed, int(self.check_adjacency), self.origin_mode, self.device)

    def validate(self) -> bool:
        c = self.cfg()
        return lib().orc_dtr_validate(ctypes.byref(c)) == 0

    def mcs_draw(self, m: int):
        c = self.cfg()
        out = np.zeros(6, dtype=np.uint32)
        lib().orc_mcs_draw(ctypes.byref(c), m, _u32(out))
        return int(out[0]), int(out[1]), tuple(int(v) for v in out[2:])

    def mcs(self, s: np.ndarray, m: int, hits: np.ndarray | None = None) -> int:
        """Apply MCS number m (0-based) to the whole lattice s in place; returns attempts.

        hits (optional, uint32 of shape (L, L)) is incremented at every attempted site.
        """
        c = self.cfg()
        stamp = None
        if self.check_adjacency:
            stamp = np.zeros(self.L * self.L, dtype=np.int32)
        n = lib().orc_dtr_mcs(_u8(s), None, ctypes.byref(c), m,
                              stamp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
                              if stamp is not None else None,
                              _u32(hits) if hits is not None else None)
        if n < 0:
            raise RuntimeError("oracle DTr emulation failed with code %d" % n)
        return n

    def mcs_window(self, s: np.ndarray, valid: np.ndarray, window, m: int) -> int:
        """Apply MCS m to a window (wx0, wy0, W, H) of the lattice.

        s and valid have shape (H, W).  Domains whose footprint is not wholly
        inside the window and valid are skipped and their footprint marked
        invalid, so every site still flagged valid afterwards holds exactly
        the value the whole-lattice run would give.
        """
        c = self.cfg(window)
        n = lib().orc_dtr_mcs(_u8(s), _u8(valid), ctypes.byref(c), m, None, None)
        if n < 0:
            raise RuntimeError("oracle DTr emulation failed with code %d" % n)
        return n


def init_flat_window(L: int, window) -> tuple:
    """Flat state of the window (wx0, wy0, W, H) and all-valid flags."""
    wx0, wy0, W, H = window
    x = (wx0 + np.arange(W)) % L
    y = (wy0 + np.arange(H)) % L
    odd = ((x[None, :] + y[:, None]) & 1).astype(np.uint8)
    return np.ascontiguousarray(odd | (odd << 1)), np.ones((H, W), dtype=np.uint8)


# --------------------------------------------------------------------------- observables
def heights(s: np.ndarray) -> np.ndarray:
    L = s.shape[0]
    h = np.zeros((L, L), dtype=np.int64)
    lib().orc_heights(_u8(s), L, _i64(h))
    return h


def _from_pair(lo: int, hi: int) -> int:
    return (int(hi) << 64) | (int(lo) & ((1 << 64) - 1))


def moments(s: np.ndarray) -> dict:
    """Exact parity-split moments {n_even, n_odd, s1_even, s1_odd, s2_even, s2_odd}."""
    out = np.zeros(10, dtype=np.int64)
    if lib().orc_moments(_u8(s), s.shape[0], _i64(out)) != 0:
        raise MemoryError
    return {
        "n_even": int(out[0]), "n_odd": int(out[1]),
        "s1_even": _from_pair(out[2], out[3]), "s1_odd": _from_pair(out[4], out[5]),
        "s2_even": _from_pair(out[6], out[7]), "s2_odd": _from_pair(out[8], out[9]),
    }


def w2_from_moments(mo: dict) -> float:
    """W^2 = <h^2> - <h>^2 over all sites (Sec. 2.1), correctly rounded."""
    n = mo["n_even"] + mo["n_odd"]
    s1 = mo["s1_even"] + mo["s1_odd"]
    s2 = mo["s2_even"] + mo["s2_odd"]
    return float(Fraction(n * s2 - s1 * s1, n * n))


def w2_sub_from_moments(mo: dict) -> float:
    """Mean of the within-parity-class variances (0 on every flat state)."""
    ve = Fraction(mo["n_even"] * mo["s2_even"] - mo["s1_even"] ** 2, mo["n_even"] ** 2)
    vo = Fraction(mo["n_odd"] * mo["s2_odd"] - mo["s1_odd"] ** 2, mo["n_odd"] ** 2)
    return float((ve + vo) / 2)


def w2(s: np.ndarray) -> float:
    return w2_from_moments(moments(s))


def cross(st: np.ndarray, ss: np.ndarray) -> int:
    out = np.zeros(2, dtype=np.int64)
    if lib().orc_cross(_u8(st), _u8(ss), st.shape[0], _i64(out)) != 0:
        raise MemoryError
    return _from_pair(out[0], out[1])


def c_h(st: np.ndarray, ss: np.ndarray) -> float:
    """C_h(t,s) = <h_t h_s> - <h_t><h_s> over sites (Sec. 2.1), correctly rounded."""
    n = st.shape[0] * st.shape[1]
    mt, ms = moments(st), moments(ss)
    s1t = mt["s1_even"] + mt["s1_odd"]
    s1s = ms["s1_even"] + ms["s1_odd"]
    return float(Fraction(n * cross(st, ss) - s1t * s1s, n * n))


def slope_overlap(st: np.ndarray, ss: np.ndarray) -> int:
    """Number of slope variables (both directions, all sites) equal to 1 in both states."""
    return int(lib().orc_slope_overlap(_u8(st), _u8(ss), st.shape[0]))


def c_s(st: np.ndarray, ss: np.ndarray) -> float:
    """Slope autocorrelation C_s(t,s) = <n_t n_s> - <n_t><n_s> over the 2 L^2
    slope variables (Sec. 2.1), with <n> = 1/2 by particle conservation;
    correctly rounded."""
    n = 2 * st.shape[0] * st.shape[1]
    return float(Fraction(slope_overlap(st, ss), n) - Fraction(1, 4))
