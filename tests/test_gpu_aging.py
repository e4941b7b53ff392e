"""The aging pipeline (Sec. 2.1): two-time autocorrelations of an ensemble of
realisations measured with the batched calls.

* exact identities at equal times: C_h(s, s) = W^2(s) (both from the same
  integer sums) and C_s(s, s) = 1/4 (every state has L^2 slope variables equal
  to 1 out of 2 L^2);
* the aging scaling of Eq. `eq:kpz_ac_C`: C_h(t, s) / C_h(s, s) depends on
  t / s only, so the curves of two waiting times coincide within their errors,
  and it decays with t / s (positive effective lambda_h / z).
"""
import numpy as np
import pytest

from paper_1705_01022_amd import aging

pytestmark = pytest.mark.gpu


def test_equal_time_identities(okpz):
    L, s = 256, 6
    ens = aging.autocorrelation(okpz, 8, L, 64, 8, okpz.BLOCK_DB, 0.95, 0.05, s, [s, s + 1, 2 * s], seed=4)
    assert np.array_equal(ens.c_h[:, 0], ens.w2[:, 0])
    assert np.all(ens.c_s[:, 0] == 0.25)
    assert np.all(ens.c_s[:, 1:] < 0.25)
    # different realisations, different surfaces
    assert len(set(ens.w2[:, 0].tolist())) > 1


def test_aging_scaling_collapse(okpz):
    L, n = 512, 128
    f = {}
    for s in (32, 64):
        ens = aging.autocorrelation(okpz, n, L, 256, 8, okpz.BLOCK_DB, 1.0, 0.0, s, [s, 2 * s, 4 * s], seed=8,
                                    stream0=1000 * s)
        x, fs, err = aging.scaling_function(ens)
        assert list(x) == [1.0, 2.0, 4.0]
        assert fs[0] == 1.0 and 1.0 > fs[1] > fs[2] > 0.0
        lam, lam_err = aging.effective_exponent(ens.times, ens.c_h, 2, 1)
        print("s=%d f(2)=%.4f+-%.4f f(4)=%.4f+-%.4f lambda_h/z(eff) = %.3f +- %.3f"
              % (s, fs[1], err[1], fs[2], err[2], -lam, lam_err))
        assert -lam > 0.0
        f[s] = (fs, err)
    for k in (1, 2):
        d = abs(f[32][0][k] - f[64][0][k])
        tol = max(3.0 * float(np.hypot(f[32][1][k], f[64][1][k])), 0.03)
        print("t/s=%d: |f_32 - f_64| = %.4f (tolerance %.4f)" % (2 ** k, d, tol))
        assert d < tol
