"""MI355X-native octahedron-model KPZ simulator (DTr domain decomposition).

Thin ctypes binding of the C ABI in ``include/okpz.h`` (library
``paper_1705_01022_amd/lib/libokpz.so``, built for gfx950 by
``paper_1705_01022_amd.build``).  Every step of the simulation runs in the
library's HIP kernels; this module only marshals arguments.  There is no CPU
fallback: if the library is missing, ``load()`` raises.

Method: Kelling, Odor, Gemming, arXiv:1705.01022 -- random-sequential updates of
the octahedron model (Sec. 2.1) parallelised by double tiling with a random
origin each MCS (DTr, Sec. 3) at device level and single-hit DT / DB / DTr at
block level (Sec. 3.1); roughness W^2 and height autocorrelation C_h (Sec. 2.1).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libokpz.so")

OK, EINVAL, ENOMEM, EHIP, EOVERFLOW, ESTATE, EWAIT = 0, -1, -2, -3, -4, -5, -6
BLOCK_DT, BLOCK_DB, BLOCK_DTR = 0, 1, 2
ORIGIN_RANDOM, ORIGIN_FIXED, ORIGIN_COARSE = 0, 1, 2
DEVICE_DT, DEVICE_DB = 0, 1
SCHEMES = {"DT": BLOCK_DT, "DB": BLOCK_DB, "DTR": BLOCK_DTR, "DTr": BLOCK_DTR}


class OkpzError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        msg = "%s failed: %s (%d)" % (what, _strerror(status), status)
        if detail:
            msg += ": " + detail
        super().__init__(msg)


class Params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_uint32),
        ("dom_x", ctypes.c_uint32),
        ("dom_y", ctypes.c_uint32),
        ("cell_x", ctypes.c_uint32),
        ("cell_y", ctypes.c_uint32),
        ("block_scheme", ctypes.c_int32),
        ("seed", ctypes.c_uint32),
        ("stream", ctypes.c_uint32),
        ("origin_mode", ctypes.c_int32),
        ("device_layer", ctypes.c_uint32),
    ]


class I128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_int64)]

    def value(self) -> int:
        return (int(self.hi) << 64) | int(self.lo)


class Moments(ctypes.Structure):
    _fields_ = [
        ("mcs", ctypes.c_uint64),
        ("n_even", ctypes.c_int64),
        ("n_odd", ctypes.c_int64),
        ("s1_even", I128),
        ("s1_odd", I128),
        ("s2_even", I128),
        ("s2_odd", I128),
        ("w2", ctypes.c_double),
        ("w2_sub", ctypes.c_double),
    ]


class Correlation(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_uint64),
        ("s", ctypes.c_uint64),
        ("s_ts", I128),
        ("s1_t", I128),
        ("s1_s", I128),
        ("c_h", ctypes.c_double),
        ("overlap", ctypes.c_int64),
        ("c_s", ctypes.c_double),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_uint64),
        ("max_members", ctypes.c_uint32),
        ("chunk_mcs", ctypes.c_uint32),
        ("threads", ctypes.c_uint32),
        ("grid", ctypes.c_uint32),
        ("use_graph", ctypes.c_int32),
        ("reserved", ctypes.c_uint32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("L", ctypes.c_uint32),
        ("n_mcs", ctypes.c_uint64),
        ("moments", Moments),
        ("t_submit", ctypes.c_double),
        ("t_start", ctypes.c_double),
        ("t_finish", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("finished", ctypes.c_uint64),
        ("queued", ctypes.c_uint64),
        ("admitted", ctypes.c_uint64),
        ("ticks", ctypes.c_uint64),
        ("attempts", ctypes.c_uint64),
        ("max_members", ctypes.c_uint64),
        ("busy_seconds", ctypes.c_double),
        ("clock", ctypes.c_double),
    ]


# name -> (restype, argtypes); the same names as include/okpz.h
_P = ctypes.c_void_p
_SIGS = {
    "okpz_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "okpz_last_error": (ctypes.c_char_p, []),
    "okpz_version": (ctypes.c_int, []),
    "okpz_validate": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
    "okpz_create": (ctypes.c_int, [ctypes.POINTER(Params), _P, ctypes.POINTER(_P)]),
    "okpz_create_external": (ctypes.c_int, [ctypes.POINTER(Params), _P, _P, ctypes.c_size_t,
                                             ctypes.POINTER(_P)]),
    "okpz_destroy": (ctypes.c_int, [_P]),
    "okpz_init_flat": (ctypes.c_int, [_P]),
    "okpz_init_from_host": (ctypes.c_int, [_P, _P, ctypes.c_uint64]),
    "okpz_run": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_double, ctypes.c_double]),
    "okpz_measure": (ctypes.c_int, [_P, ctypes.POINTER(Moments)]),
    "okpz_measure_noalloc": (ctypes.c_int, [_P, ctypes.c_uint32, _P, _P, ctypes.POINTER(Moments)]),
    "okpz_snapshot": (ctypes.c_int, [_P]),
    "okpz_autocorr": (ctypes.c_int, [_P, ctypes.POINTER(Correlation)]),
    "okpz_observe": (ctypes.c_int, [_P, ctypes.POINTER(Moments), ctypes.POINTER(Correlation)]),
    "okpz_get_sites": (ctypes.c_int, [_P, _P]),
    "okpz_checkpoint_size": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "okpz_save": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_size_t]),
    "okpz_load": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "okpz_get_window": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, _P]),
    "okpz_set_window": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, _P]),
    "okpz_get_heights": (ctypes.c_int, [_P, _P]),
    "okpz_get_words": (ctypes.c_int, [_P, _P]),
    "okpz_device_words": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_size_t)]),
    "okpz_get_mcs": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64)]),
    "okpz_get_params": (ctypes.c_int, [_P, ctypes.POINTER(Params)]),
    "okpz_set_threads": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "okpz_sync": (ctypes.c_int, [_P]),
    "okpz_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "okpz_get_timing": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_uint64),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "okpz_philox": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, _P, _P, ctypes.c_size_t]),
    "okpz_batch_create": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "okpz_batch_destroy": (ctypes.c_int, [_P]),
    "okpz_batch_add": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int32)]),
    "okpz_batch_remove": (ctypes.c_int, [_P, ctypes.c_int32]),
    "okpz_batch_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint32)]),
    "okpz_batch_config": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]),
    "okpz_batch_wait_set": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_uint32, _P]),
    "okpz_batch_run": (ctypes.c_int, [_P, _P, _P, _P]),
    "okpz_batch_sync": (ctypes.c_int, [_P]),
    "okpz_batch_observe": (ctypes.c_int, [_P, ctypes.POINTER(Moments), ctypes.POINTER(Correlation)]),
    "okpz_batch_snapshot": (ctypes.c_int, [_P]),
    "okpz_batch_series": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, _P,
                                          ctypes.POINTER(Moments), ctypes.POINTER(Correlation)]),
    "okpz_batch_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "okpz_batch_get_timing": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_uint64),
                                              ctypes.POINTER(ctypes.c_uint64)]),
    "okpz_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), _P, ctypes.POINTER(_P)]),
    "okpz_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(Params), ctypes.c_uint64, ctypes.c_double,
                                           ctypes.c_double, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "okpz_server_poll": (ctypes.c_int, [_P, ctypes.POINTER(Result), ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_uint32)]),
    "okpz_server_drain": (ctypes.c_int, [_P, ctypes.c_double]),
    "okpz_server_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(ServerStats)]),
    "okpz_server_destroy": (ctypes.c_int, [_P]),
}

_lib = None


def load():
    """Load the HIP library; raise if it has not been built.

    torch is imported first when it is installed: its libraries load the HIP
    runtime it ships with, and the library then binds to that same runtime (its
    libamdhip64.so.7 dependency is satisfied by the already-loaded copy), so one
    process never holds two HIP runtimes and torch tensors and streams can be
    handed to the library.
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError("HIP library %s is missing: run `python -m paper_1705_01022_amd.build` "
                              "(there is no CPU fallback)" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _strerror(status: int) -> str:
    try:
        return load().okpz_strerror(status).decode()
    except Exception:  # noqa: BLE001 - message formatting only
        return "status"


def _check(status: int, what: str, explained: bool = False):
    """Raise on a failed status; the HIP error text (or, for calls that set
    one with every error, ``explained``) goes into the message."""
    if status != OK:
        detail = load().okpz_last_error().decode() if (status == EHIP or explained) else ""
        raise OkpzError(status, what, detail)


def _ptr(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


def params(L, Dx, Dy, Cx, Cy, scheme=BLOCK_DT, seed=1, stream=0, origin_mode=ORIGIN_RANDOM,
           device_layer=DEVICE_DT) -> Params:
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    return Params(L, Dx, Dy, Cx, Cy, scheme, seed, stream, origin_mode, device_layer)


def validate(prm: Params) -> int:
    n = ctypes.c_size_t(0)
    st = load().okpz_validate(ctypes.byref(prm), ctypes.byref(n))
    return n.value if st == OK else st


def _to_int(v: I128) -> int:
    return v.value()


class Lattice:
    """One octahedron-model lattice resident on the GPU."""

    def __init__(self, L, Dx, Dy, Cx, Cy, scheme=BLOCK_DT, seed=1, stream=0,
                 origin_mode=ORIGIN_RANDOM, hip_stream=None, device_buffer=None, device_layer=DEVICE_DT):
        lib = load()
        self.prm = params(L, Dx, Dy, Cx, Cy, scheme, seed, stream, origin_mode, device_layer)
        self.L = L
        h = ctypes.c_void_p()
        s = ctypes.c_void_p(hip_stream) if hip_stream else None
        if device_buffer is not None:
            ptr, nbytes = device_buffer
            _check(lib.okpz_create_external(ctypes.byref(self.prm), s, ctypes.c_void_p(ptr), nbytes,
                                            ctypes.byref(h)), "okpz_create_external")
        else:
            _check(lib.okpz_create(ctypes.byref(self.prm), s, ctypes.byref(h)), "okpz_create")
        self._h = h

    # -- lifecycle
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().okpz_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- state
    def init_flat(self):
        _check(load().okpz_init_flat(self._h), "okpz_init_flat")

    def init_from_host(self, sites: np.ndarray, mcs: int = 0):
        s = np.ascontiguousarray(sites, dtype=np.uint8)
        assert s.shape == (self.L, self.L)
        _check(load().okpz_init_from_host(self._h, _ptr(s), mcs), "okpz_init_from_host")

    @property
    def mcs(self) -> int:
        v = ctypes.c_uint64()
        _check(load().okpz_get_mcs(self._h, ctypes.byref(v)), "okpz_get_mcs")
        return v.value

    def run(self, n_mcs: int, p: float, q: float):
        _check(load().okpz_run(self._h, n_mcs, p, q), "okpz_run")

    def set_threads(self, threads: int):
        """Device-step workgroup size in lanes (64, 128, 256 or 512; 0 = automatic); results do not change."""
        _check(load().okpz_set_threads(self._h, threads), "okpz_set_threads")

    def sync(self):
        _check(load().okpz_sync(self._h), "okpz_sync")

    # -- observables
    def measure(self) -> dict:
        m = Moments()
        _check(load().okpz_measure(self._h, ctypes.byref(m)), "okpz_measure")
        return _moments_dict(m)

    def observe(self, with_autocorr: bool = True):
        """Moments and (optionally) C_h from one pass; returns (moments, corr or None)."""
        m, c = Moments(), Correlation()
        _check(load().okpz_observe(self._h, ctypes.byref(m), ctypes.byref(c) if with_autocorr else None),
               "okpz_observe")
        return _moments_dict(m), (_corr_dict(c) if with_autocorr else None)

    def snapshot(self):
        _check(load().okpz_snapshot(self._h), "okpz_snapshot")

    def autocorr(self) -> dict:
        c = Correlation()
        _check(load().okpz_autocorr(self._h, ctypes.byref(c)), "okpz_autocorr")
        return _corr_dict(c)

    # -- checkpoint / resume
    def save(self, with_snapshot: bool = False) -> np.ndarray:
        """The state (and snapshot) as a checkpoint blob (uint8 array)."""
        n = ctypes.c_size_t()
        _check(load().okpz_checkpoint_size(self._h, int(with_snapshot), ctypes.byref(n)), "okpz_checkpoint_size")
        out = np.empty(n.value, dtype=np.uint8)
        _check(load().okpz_save(self._h, int(with_snapshot), _ptr(out), out.size), "okpz_save")
        return out

    def load(self, blob):
        """Restore a checkpoint written by :meth:`save` of a lattice with the
        same parameters."""
        b = np.ascontiguousarray(np.frombuffer(blob, dtype=np.uint8) if isinstance(blob, (bytes, bytearray))
                                 else blob, dtype=np.uint8)
        _check(load().okpz_load(self._h, _ptr(b), b.size), "okpz_load")

    # -- export / import
    def sites(self) -> np.ndarray:
        out = np.zeros((self.L, self.L), dtype=np.uint8)
        _check(load().okpz_get_sites(self._h, _ptr(out)), "okpz_get_sites")
        return out

    def window(self, x0: int, y0: int, w: int, h: int) -> np.ndarray:
        out = np.zeros((h, w), dtype=np.uint8)
        _check(load().okpz_get_window(self._h, x0, y0, w, h, _ptr(out)), "okpz_get_window")
        return out

    def set_window(self, x0: int, y0: int, sites: np.ndarray):
        s = np.ascontiguousarray(sites, dtype=np.uint8)
        h, w = s.shape
        _check(load().okpz_set_window(self._h, x0, y0, w, h, _ptr(s)), "okpz_set_window")

    def heights(self) -> np.ndarray:
        out = np.zeros((self.L, self.L), dtype=np.int32)
        _check(load().okpz_get_heights(self._h, _ptr(out)), "okpz_get_heights")
        return out

    def words(self) -> np.ndarray:
        out = np.zeros(self.L * self.L // 16, dtype=np.uint32)
        _check(load().okpz_get_words(self._h, _ptr(out)), "okpz_get_words")
        return out

    def device_words(self):
        p, n = ctypes.c_void_p(), ctypes.c_size_t()
        _check(load().okpz_device_words(self._h, ctypes.byref(p), ctypes.byref(n)),
               "okpz_device_words")
        return p.value, n.value

    # -- timing
    def timing(self, enable: bool = True):
        _check(load().okpz_timing(self._h, int(enable)), "okpz_timing")

    def get_timing(self) -> dict:
        sm, mm = ctypes.c_double(), ctypes.c_double()
        sn, mn = ctypes.c_uint64(), ctypes.c_uint64()
        _check(load().okpz_get_timing(self._h, ctypes.byref(sm), ctypes.byref(sn), ctypes.byref(mm),
                                      ctypes.byref(mn)), "okpz_get_timing")
        return {"step_ms": sm.value, "step_launches": sn.value,
                "measure_ms": mm.value, "measure_launches": mn.value}


def _moments_dict(m) -> dict:
    return {"mcs": m.mcs, "n_even": m.n_even, "n_odd": m.n_odd,
            "s1_even": _to_int(m.s1_even), "s1_odd": _to_int(m.s1_odd),
            "s2_even": _to_int(m.s2_even), "s2_odd": _to_int(m.s2_odd),
            "w2": m.w2, "w2_sub": m.w2_sub}


def measure_noalloc(dev_words: int, L: int, dev_totals: int, hip_stream: int = 0, synchronous: bool = True):
    """Exact height moments of a packed lattice in caller-owned device memory
    without any allocation (``okpz_measure_noalloc``).  ``dev_words``,
    ``dev_totals`` (96 bytes, 8-byte aligned) and ``hip_stream`` are raw device
    pointers / a raw hipStream_t.  With ``synchronous`` the call waits and
    returns the moments (mcs = 0); otherwise it only enqueues the kernels and
    returns None (the totals land in ``dev_totals``)."""
    m = Moments()
    _check(load().okpz_measure_noalloc(ctypes.c_void_p(dev_words), L,
                                       ctypes.c_void_p(hip_stream) if hip_stream else None,
                                       ctypes.c_void_p(dev_totals), ctypes.byref(m) if synchronous else None),
           "okpz_measure_noalloc", explained=True)
    return _moments_dict(m) if synchronous else None


def batch_wait_set(L, Dx, Dy, tile, new_tiling=False, ox=0, oy=0, oxp=0, oyp=0) -> tuple:
    """Tiles of the previous device step that a batch work item waits for
    (host-only call): (first column, columns, first row, rows)."""
    out = (ctypes.c_uint32 * 4)()
    _check(load().okpz_batch_wait_set(L, Dx, Dy, tile, int(bool(new_tiling)), ox, oy, oxp, oyp, out),
           "okpz_batch_wait_set")
    return tuple(out)


def _corr_dict(c) -> dict:
    return {"t": c.t, "s": c.s, "s_ts": _to_int(c.s_ts), "s1_t": _to_int(c.s1_t),
            "s1_s": _to_int(c.s1_s), "c_h": c.c_h, "overlap": c.overlap, "c_s": c.c_s}


class Batch:
    """Many lattices advanced together by one persistent kernel launch per run.

    Members are ordinary :class:`Lattice` objects on the batch's HIP stream
    (``Batch.lattice`` creates one); each keeps its full single-lattice API.
    ``hip_stream``: a raw hipStream_t; by default the batch creates its own
    torch stream (graph capture needs a non-null stream).
    """

    def __init__(self, hip_stream=None):
        lib = load()
        self._torch_stream = None
        if hip_stream is None:
            import torch

            self._torch_stream = torch.cuda.Stream()
            hip_stream = self._torch_stream.cuda_stream
        self.hip_stream = hip_stream
        h = ctypes.c_void_p()
        _check(lib.okpz_batch_create(ctypes.c_void_p(hip_stream) if hip_stream else None, ctypes.byref(h)),
               "okpz_batch_create")
        self._h = h
        self.members = {}

    def lattice(self, L, Dx, Dy, Cx, Cy, scheme=BLOCK_DT, seed=1, stream=0, origin_mode=ORIGIN_RANDOM,
                add=True) -> Lattice:
        """A new lattice on the batch's stream (added as a member unless add=False)."""
        lat = Lattice(L, Dx, Dy, Cx, Cy, scheme, seed, stream, origin_mode, hip_stream=self.hip_stream)
        if add:
            self.add(lat)
        return lat

    def add(self, lat: Lattice) -> int:
        slot = ctypes.c_int32()
        _check(load().okpz_batch_add(self._h, lat._h, ctypes.byref(slot)), "okpz_batch_add")
        self.members[slot.value] = lat
        lat.slot = slot.value
        return slot.value

    def remove(self, slot: int):
        _check(load().okpz_batch_remove(self._h, slot), "okpz_batch_remove")
        self.members.pop(slot, None)

    @property
    def size(self) -> int:
        n = ctypes.c_uint32()
        _check(load().okpz_batch_size(self._h, ctypes.byref(n)), "okpz_batch_size")
        return n.value

    def config(self, threads: int = 0, grid: int = 0, use_graph: bool = True):
        """Launch shape only (results do not depend on it)."""
        _check(load().okpz_batch_config(self._h, threads, grid, int(use_graph)), "okpz_batch_config")
        self._config = (threads, grid, use_graph)

    def run(self, n_mcs, p, q):
        """n_mcs, p, q: dicts slot -> value or sequences indexed by slot (0 MCS = idle)."""
        n = self.size
        nm = np.zeros(n, dtype=np.uint64)
        pp = np.zeros(n, dtype=np.float64)
        qq = np.zeros(n, dtype=np.float64)
        for arr, src in ((nm, n_mcs), (pp, p), (qq, q)):
            if isinstance(src, dict):
                for k, v in src.items():
                    arr[k] = v
            elif np.isscalar(src):
                arr[[k for k in self.members]] = src
            else:
                arr[:len(src)] = src
        _check(load().okpz_batch_run(self._h, _ptr(nm), _ptr(pp), _ptr(qq)), "okpz_batch_run")

    def sync(self):
        _check(load().okpz_batch_sync(self._h), "okpz_batch_sync")

    def _rates(self, p, q):
        n = self.size
        pp = np.zeros(n, dtype=np.float64)
        qq = np.zeros(n, dtype=np.float64)
        for arr, src in ((pp, p), (qq, q)):
            if isinstance(src, dict):
                for k, v in src.items():
                    arr[k] = v
            elif np.isscalar(src):
                arr[[k for k in self.members]] = src
            else:
                arr[:len(src)] = src
        return pp, qq

    def snapshot(self):
        """Snapshot of every member (reference time s of C_h(t, s))."""
        _check(load().okpz_batch_snapshot(self._h), "okpz_batch_snapshot")

    def observe(self, with_autocorr: bool = False) -> dict:
        """Moments (and C_h, C_s against the snapshots) of every member in
        three launches: {slot: (moments, corr or None)}."""
        n = self.size
        m = (Moments * max(n, 1))()
        c = (Correlation * max(n, 1))() if with_autocorr else None
        _check(load().okpz_batch_observe(self._h, m, c), "okpz_batch_observe")
        return {s: (_moments_dict(m[s]), _corr_dict(c[s]) if with_autocorr else None) for s in self.members}

    def series(self, times, p, q, with_autocorr: bool = False) -> list:
        """Advance every member to each of ``times`` (MCS from now, non-
        decreasing) and observe all members there; one entry per time:
        {slot: (moments, corr or None)}."""
        n = self.size
        t = np.ascontiguousarray(times, dtype=np.uint64)
        pp, qq = self._rates(p, q)
        k = len(t)
        m = (Moments * max(n * k, 1))()
        c = (Correlation * max(n * k, 1))() if with_autocorr else None
        _check(load().okpz_batch_series(self._h, _ptr(t), k, _ptr(pp), _ptr(qq), m, c), "okpz_batch_series")
        return [{s: (_moments_dict(m[i * n + s]), _corr_dict(c[i * n + s]) if with_autocorr else None)
                 for s in self.members} for i in range(k)]

    def timing(self, enable: bool = True):
        _check(load().okpz_batch_timing(self._h, int(enable)), "okpz_batch_timing")

    def get_timing(self) -> dict:
        ms, nl, na = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(load().okpz_batch_get_timing(self._h, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(na)),
               "okpz_batch_get_timing")
        return {"ms": ms.value, "launches": nl.value, "attempts": na.value}

    def tune(self, n_mcs, p, q, candidates=None) -> dict:
        """Autotune the launch shape on real work: run ``n_mcs`` (per member)
        under each candidate (threads, grid fraction, graph) and keep the
        fastest.  Every candidate's MCS really advance the members (results do
        not depend on the shape).  Returns {candidate: ms} and the choice."""
        if candidates is None:
            candidates = [(256, 1.0, True), (128, 1.0, True), (512, 1.0, True), (256, 0.5, True),
                          (256, 1.0, False)]
        full = self._full_grid()
        times = {}
        for threads, frac, graph in candidates:
            grid = max(1, int(full * frac)) if frac < 1.0 else 0
            self.config(threads, grid, graph)
            self.run(n_mcs, p, q)  # warm (captures the graph)
            self.sync()
            self.timing(True)
            self.run(n_mcs, p, q)
            self.sync()
            times[(threads, frac, graph)] = self.get_timing()["ms"]
            self.timing(False)
        best = min(times, key=times.get)
        threads, frac, graph = best
        self.config(threads, max(1, int(full * frac)) if frac < 1.0 else 0, graph)
        return {"times_ms": times, "best": best}

    @staticmethod
    def _full_grid() -> int:
        import torch

        return torch.cuda.get_device_properties(0).multi_processor_count * 4

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().okpz_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Request loop with continuous batching (native worker thread).

    ``submit`` queues a simulation request and returns its id; ``poll``
    returns finished results (dicts with the final moments, the final sites
    if asked for, and submit/start/finish times on the server clock).
    """

    def __init__(self, hbm_budget=64 << 30, max_members=1024, chunk_mcs=64, threads=0, grid=0,
                 use_graph=True, hip_stream=None):
        lib = load()
        self._torch_stream = None
        if hip_stream is None:
            import torch

            self._torch_stream = torch.cuda.Stream()
            hip_stream = self._torch_stream.cuda_stream
        cfg = ServerConfig(hbm_budget, max_members, chunk_mcs, threads, grid, int(use_graph), 0)
        h = ctypes.c_void_p()
        _check(lib.okpz_server_create(ctypes.byref(cfg), ctypes.c_void_p(hip_stream), ctypes.byref(h)),
               "okpz_server_create")
        self._h = h
        self._sites = {}  # id -> host buffer the worker writes the final sites into

    def submit(self, L, Dx, Dy, Cx, Cy, scheme, seed, stream, n_mcs, p, q, want_sites=False) -> int:
        prm = params(L, Dx, Dy, Cx, Cy, scheme, seed, stream)
        buf = np.zeros((L, L), dtype=np.uint8) if want_sites else None
        rid = ctypes.c_uint64()
        _check(load().okpz_server_submit(self._h, ctypes.byref(prm), n_mcs, p, q,
                                         _ptr(buf) if buf is not None else None, ctypes.byref(rid)),
               "okpz_server_submit")
        if buf is not None:
            self._sites[rid.value] = buf
        return rid.value

    def poll(self, max_results=256) -> list:
        arr = (Result * max_results)()
        n = ctypes.c_uint32()
        _check(load().okpz_server_poll(self._h, arr, max_results, ctypes.byref(n)), "okpz_server_poll")
        out = []
        for r in arr[:n.value]:
            d = {"id": r.id, "status": r.status, "L": r.L, "n_mcs": r.n_mcs,
                 "moments": _moments_dict(r.moments), "t_submit": r.t_submit, "t_start": r.t_start,
                 "t_finish": r.t_finish}
            if r.id in self._sites:
                d["sites"] = self._sites.pop(r.id)
            out.append(d)
        return out

    def drain(self, timeout=600.0):
        _check(load().okpz_server_drain(self._h, timeout), "okpz_server_drain")

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().okpz_server_get_stats(self._h, ctypes.byref(st)), "okpz_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().okpz_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def philox(k0: int, k1: int, counters: np.ndarray) -> np.ndarray:
    """Device Philox4x32-10 blocks for an (n, 4) uint32 array of counters."""
    c = np.ascontiguousarray(counters, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros_like(c)
    _check(load().okpz_philox(k0, k1, _ptr(c), _ptr(out), c.shape[0]), "okpz_philox")
    return out


def exported_symbols() -> list:
    return sorted(_SIGS)


def hip_runtime_paths() -> list:
    """Paths of the HIP runtime libraries mapped into this process."""
    out = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                out.add(line.split()[-1])
    return sorted(out)
