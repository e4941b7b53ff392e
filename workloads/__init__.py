"""Seeded synthetic workloads for the octahedron-model simulations.

This module only describes inputs: lattice sizes, decomposition parameters,
rates, seeds, and the random composition of batched and served work.  It holds
none of the method's arithmetic, so both the GPU tests / benchmark and the CPU
oracle can draw their inputs from it.  Every input of the method is the flat
zig-zag surface plus the counter-based random stream keyed by (seed, stream).

The paper (Kelling, Odor, Gemming, arXiv:1705.01022) runs the octahedron model
on L = 2^12 .. 2^17 lattices from a flat start, at p = 1, q = 0 (KPZ), with DTr
at device level and single-hit DT or DB on TC=1,1 (8x8-site) cells at block
level (Secs. 3.1, 4.1-4.3).  Device domains of 256 x 256 sites are this
build's reading of the 48 kB local-memory constraint the paper states
(Sec. 2.2); they are a fixed physics parameter, not a tuning knob.
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict

import numpy as np

DT, DB, DTR = 0, 1, 2
SCHEME_NAMES = {DT: "DTrDT", DB: "DTrDB", DTR: "DTrDTr"}


@dataclass(frozen=True)
class Workload:
    name: str
    L: int
    Dx: int
    Dy: int
    Cx: int
    Cy: int
    scheme: int
    p: float
    q: float
    n_mcs: int
    seed: int = 1
    streams: tuple = (0,)
    measure_times: tuple = ()
    snapshot_at: int | None = None

    def params(self, stream: int | None = None) -> dict:
        return dict(L=self.L, Dx=self.Dx, Dy=self.Dy, Cx=self.Cx, Cy=self.Cy, scheme=self.scheme,
                    seed=self.seed, stream=self.streams[0] if stream is None else stream)

    def as_dict(self) -> dict:
        return asdict(self)


def log_times(t_max: int, per_decade: int = 10) -> tuple:
    """{0} and unique round(10^(i/per_decade)) up to t_max."""
    out = {0}
    i = 0
    while True:
        t = int(round(10 ** (i / per_decade)))
        if t > t_max:
            break
        out.add(t)
        i += 1
    return tuple(sorted(out))


# Small case: L=64, every MCS measured; the oracle finishes it in seconds.
SMALL = Workload("octahedron L=64 flat start, p=1 q=0, 1000 MCS", L=64, Dx=16, Dy=16, Cx=8, Cy=8,
                 scheme=DT, p=1.0, q=0.0, n_mcs=1000, measure_times=tuple(range(1001)))

# Single lattice L=4096 (4 MiB packed), DTrDT, 10^4 MCS, 64 streams.
L4096 = Workload("octahedron L=4096 DTrDT p=1 q=0", L=4096, Dx=256, Dy=256, Cx=8, Cy=8, scheme=DT,
                 p=1.0, q=0.0, n_mcs=10_000, streams=tuple(range(64)),
                 measure_times=log_times(10_000))

# Single lattice L=2^17 (4 GiB packed), DTrDB, p=0.95 q=0.05, C_h at s=1000.
L131072 = Workload("octahedron L=131072 DTrDB p=0.95 q=0.05", L=1 << 17, Dx=256, Dy=256, Cx=8,
                   Cy=8, scheme=DB, p=0.95, q=0.05, n_mcs=100_000,
                   measure_times=log_times(100_000), snapshot_at=1000)


@dataclass
class BatchMember:
    L: int
    p: float
    q: float
    stream: int
    Dx: int
    Dy: int
    Cx: int = 8
    Cy: int = 8
    scheme: int = DT


def batched_composition(n: int = 512, seed: int = 1) -> list:
    """512 realizations: L uniform over {256, 512, 1024, 2048}; (p, q) = (1, 0)
    or (1/2, 1/2) with probability 1/2 each; streams 0..n-1; D = min(256, L/2)."""
    rng = np.random.default_rng(seed)
    Ls = rng.choice([256, 512, 1024, 2048], size=n)
    kinds = rng.integers(0, 2, size=n)
    out = []
    for i in range(n):
        L = int(Ls[i])
        p, q = (1.0, 0.0) if kinds[i] == 0 else (0.5, 0.5)
        D = min(256, L // 2)
        out.append(BatchMember(L=L, p=p, q=q, stream=i, Dx=D, Dy=D))
    return out


@dataclass
class Request:
    rid: int
    arrival: float
    L: int
    n_mcs: int
    p: float
    q: float
    Dx: int
    Dy: int
    Cx: int = 8
    Cy: int = 8
    scheme: int = DB


def serving_requests(n: int = 2000, rate: float = 200.0, seed: int = 1) -> list:
    """Poisson arrivals at `rate` per second; L = 2^U{9..13}; MCS in {10^3, 10^4}
    with probability 1/2 each; p ~ U[0.5, 1], q = 1 - p; stream = request id."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps)
    Ls = 2 ** rng.integers(9, 14, size=n)
    mcs = np.where(rng.integers(0, 2, size=n) == 0, 1000, 10_000)
    ps = rng.uniform(0.5, 1.0, size=n)
    out = []
    for i in range(n):
        L = int(Ls[i])
        D = min(256, L // 2)
        out.append(Request(rid=i, arrival=float(arrivals[i]), L=L, n_mcs=int(mcs[i]),
                           p=float(ps[i]), q=float(1.0 - ps[i]), Dx=D, Dy=D))
    return out
