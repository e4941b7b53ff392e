"""Ensemble observables of the growth and aging regimes (Sec. 2.1): the
roughness W^2(t) and the two-time autocorrelations C_h(t, s), C_s(t, s) of
many realisations run together in one batch, and effective exponents
(Eq. `eq:effexp`) with their statistical errors.

Everything on the device goes through the batch calls of the library
(``Batch.series``, ``Batch.snapshot``): every measurement time costs three
launches for the whole ensemble.  This module only arranges the runs and does
the ensemble statistics on the host.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def log_times(t_max: int, per_decade: int = 10, t_min: int = 1) -> list:
    """Measurement times t_min <= t <= t_max, about per_decade per decade:
    the distinct values of round(10^(i / per_decade)) (the log grid of the
    roughness and autocorrelation curves)."""
    out, i = [], 0
    while True:
        t = int(round(10 ** (i / per_decade)))
        if t > t_max:
            break
        if t >= t_min and (not out or t != out[-1]):
            out.append(t)
        i += 1
    return out


@dataclass
class Ensemble:
    """Per-realisation series: rows are realisations, columns measurement times."""
    times: list
    w2: np.ndarray
    s: int | None = None
    c_h: np.ndarray | None = None
    c_s: np.ndarray | None = None
    params: dict = field(default_factory=dict)


def _batch(okpz, n, L, D, C, scheme, seed, stream0, origin_mode):
    b = okpz.Batch()
    lats = [b.lattice(L, D, D, C, C, scheme, seed=seed, stream=stream0 + r, origin_mode=origin_mode)
            for r in range(n)]
    return b, lats


def _close(b, lats):
    b.close()
    for lat in lats:
        lat.close()


def roughness(okpz, n: int, L: int, D: int, C: int, scheme, p: float, q: float, times, seed: int = 1,
              stream0: int = 0, origin_mode=None) -> Ensemble:
    """W^2 at each of ``times`` (MCS from the flat state, non-decreasing) for n
    realisations (streams stream0 .. stream0 + n - 1)."""
    om = okpz.ORIGIN_RANDOM if origin_mode is None else origin_mode
    b, lats = _batch(okpz, n, L, D, C, scheme, seed, stream0, om)
    try:
        series = b.series(list(times), p, q)
    finally:
        _close(b, lats)
    w2 = np.array([[obs[r][0]["w2"] for r in range(n)] for obs in series]).T
    return Ensemble(list(times), w2, params=dict(n=n, L=L, D=D, C=C, scheme=scheme, p=p, q=q, seed=seed))


def autocorrelation(okpz, n: int, L: int, D: int, C: int, scheme, p: float, q: float, s: int, times,
                    seed: int = 1, stream0: int = 0, origin_mode=None) -> Ensemble:
    """Run n realisations to the waiting time s, take the snapshot, and
    measure W^2(t), C_h(t, s) and C_s(t, s) at each of ``times`` (absolute
    MCS, all >= s, non-decreasing)."""
    if any(t < s for t in times):
        raise ValueError("measurement times must not precede the waiting time")
    om = okpz.ORIGIN_RANDOM if origin_mode is None else origin_mode
    b, lats = _batch(okpz, n, L, D, C, scheme, seed, stream0, om)
    try:
        b.run([s] * n, p, q)
        b.snapshot()
        series = b.series([t - s for t in times], p, q, with_autocorr=True)
    finally:
        _close(b, lats)
    w2 = np.array([[obs[r][0]["w2"] for r in range(n)] for obs in series]).T
    ch = np.array([[obs[r][1]["c_h"] for r in range(n)] for obs in series]).T
    cs = np.array([[obs[r][1]["c_s"] for r in range(n)] for obs in series]).T
    return Ensemble(list(times), w2, s, ch, cs,
                    params=dict(n=n, L=L, D=D, C=C, scheme=scheme, p=p, q=q, seed=seed))


def mean_err(x: np.ndarray) -> tuple:
    """Ensemble mean of each column and its standard error."""
    n = x.shape[0]
    return x.mean(axis=0), x.std(axis=0, ddof=1) / math.sqrt(n)


def effective_exponent(times, series: np.ndarray, i: int, j: int, power: float = 1.0) -> tuple:
    """Effective exponent (Eq. `eq:effexp`) of E = <X>^power between
    times[i] and times[j] (X the columns of ``series``, realisations in rows):
    (ln E(t_i) - ln E(t_j)) / (ln t_i - ln t_j), with its standard error from
    the two sample means (delta method, covariance of the two means taken from
    the realisations).  power = 1/2 turns W^2 into W (beta_eff)."""
    n = series.shape[0]
    mi, mj = series[:, i].mean(), series[:, j].mean()
    span = math.log(times[i] / times[j])
    e = power * math.log(mi / mj) / span
    cov = np.cov(series[:, i], series[:, j]) / n
    g = np.array([power / mi, -power / mj])
    return e, math.sqrt(float(g @ cov @ g)) / abs(span)


def scaling_function(ens: Ensemble) -> tuple:
    """f(t/s) = <C_h(t, s)> / <C_h(s, s)> (s-independent in the aging regime,
    Eq. `eq:kpz_ac_C`), with its standard error (delta method).  The first
    measurement time must be s."""
    if ens.c_h is None or ens.times[0] != ens.s:
        raise ValueError("needs C_h with the waiting time as first measurement time")
    n = ens.c_h.shape[0]
    m0 = ens.c_h[:, 0].mean()
    f, err = [], []
    for k in range(len(ens.times)):
        mk = ens.c_h[:, k].mean()
        cov = np.cov(ens.c_h[:, k], ens.c_h[:, 0]) / n
        g = np.array([1.0 / m0, -mk / m0 ** 2])
        f.append(mk / m0)
        err.append(math.sqrt(max(float(g @ cov @ g), 0.0)))
    return np.array([t / ens.s for t in ens.times]), np.array(f), np.array(err)
