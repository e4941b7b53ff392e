"""Host-side statistics of the aging pipeline (no GPU): the log time grid and
the effective exponents of Eq. `eq:effexp` on synthetic ensembles whose
answer is known in closed form."""
import math

import numpy as np

from paper_1705_01022_amd import aging


def test_log_times_grid():
    t = aging.log_times(1000)
    assert t[:10] == [1, 2, 3, 4, 5, 6, 8, 10, 13, 16]
    assert t[-1] == 1000 and all(a < b for a, b in zip(t, t[1:]))
    assert aging.log_times(100, per_decade=1) == [1, 10, 100]
    assert aging.log_times(1000, t_min=50)[0] == 50


def test_effective_exponent_of_a_power_law():
    # noiseless ensemble W^2 = 3 t^(2 beta): beta_eff = beta exactly, zero error
    times = [4, 8, 16, 32]
    beta = 0.2414
    w2 = np.tile([3.0 * t ** (2 * beta) for t in times], (5, 1))
    b, e = aging.effective_exponent(times, w2, 3, 1, power=0.5)
    assert math.isclose(b, beta, rel_tol=1e-12) and e < 1e-12
    # order of the two times does not matter
    b2, _ = aging.effective_exponent(times, w2, 1, 3, power=0.5)
    assert math.isclose(b, b2, rel_tol=1e-12)


def test_effective_exponent_error_matches_sampling():
    # independent log-normal noise of relative size sigma at two times: the
    # delta-method error of the exponent is sigma * sqrt(2 / n) / ln(t_i / t_j)
    rng = np.random.default_rng(7)
    n, sigma = 4000, 0.05
    times = [10, 100]
    x = np.column_stack([np.exp(rng.normal(0, sigma, n)) * t for t in times])
    e, err = aging.effective_exponent(times, x, 1, 0)
    assert abs(e - 1.0) < 4 * err
    assert math.isclose(err, sigma * math.sqrt(2.0 / n) / math.log(10.0), rel_tol=0.1)


def test_scaling_function_closed_form():
    # C_h(t, s) = s^(2 beta) (t/s)^(-lambda/z) for every realisation: f(x) = x^(-lambda/z)
    s, lz = 16, 0.8
    times = [16, 32, 64]
    ch = np.tile([s ** 0.48 * (t / s) ** (-lz) for t in times], (4, 1))
    ens = aging.Ensemble(times, ch.copy(), s, ch, None)
    x, f, err = aging.scaling_function(ens)
    assert list(x) == [1.0, 2.0, 4.0]
    assert np.allclose(f, [1.0, 2.0 ** -lz, 4.0 ** -lz]) and np.all(err < 1e-12)
    lam, _ = aging.effective_exponent(times, ch, 2, 1)
    assert math.isclose(-lam, lz, rel_tol=1e-12)
