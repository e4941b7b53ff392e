"""Pin the sequential RS oracle against the exact master equation at L = 4.

Sequential RS (Sec. 1; the CPU reference of Sec. 4.3) picks each attempt's
site uniformly from the whole lattice.  On the 4x4 torus the 990 states make
the exact distribution after t MCS computable: P_t = P_0 T^(16 t) with T the
one-attempt transition matrix built from the height rule.  Monte Carlo means
of W^2 from the oracle must lie within 3 standard errors of the exact values
(12 comparisons; deterministic seeds).
"""
import numpy as np
import pytest

from l4_states import StateSpace, w2_of_heights, w2_sub_of_heights


@pytest.fixture(scope="module")
def space():
    return StateSpace(4)


@pytest.mark.parametrize("p,q", [(1.0, 0.0), (0.5, 0.5)])
def test_seq_rs_matches_master_equation(orc, space, p, q):
    T = space.attempt_matrix(p, q)
    M = np.linalg.matrix_power(T, 16)
    W = np.array([w2_of_heights(h) for h in space.heights])
    Ws = np.array([w2_sub_of_heights(h) for h in space.heights])
    P = np.zeros(len(space))
    P[space.flat_index()] = 1.0
    exact = []
    for _ in range(3):
        P = P @ M
        exact.append((P @ W, P @ Ws, P @ (W * W), P @ (Ws * Ws)))
    n = 20000
    samples = np.zeros((n, 3, 2))
    for r in range(n):
        sim = orc.SeqRS(4, p, q, seed=99, stream=r)
        for t in range(3):
            sim.run(1)
            mo = orc.moments(sim.s)
            samples[r, t] = orc.w2_from_moments(mo), orc.w2_sub_from_moments(mo)
    for t in range(3):
        for j in range(2):
            mean = samples[:, t, j].mean()
            var = exact[t][2 + j] - exact[t][j] ** 2
            se = np.sqrt(var / n)
            assert abs(mean - exact[t][j]) < 3 * se, (t, j, mean, exact[t][j], se)


def test_uniform_law_stationary_exact(space):
    # for p = q every per-site kernel is symmetric, so uniform is stationary
    T = space.attempt_matrix(0.3, 0.3)
    u = np.full(len(space), 1.0 / len(space))
    assert np.max(np.abs(u @ T - u)) < 1e-15


def test_seq_rs_uniform_when_p_equals_q(orc, space):
    # long chain, sampled every 4 MCS: chi-square against the uniform law
    sim = orc.SeqRS(4, 0.5, 0.5, seed=5, stream=1)
    sim.run(50)
    counts = np.zeros(len(space))
    n = 60000
    for _ in range(n):
        sim.run(4)
        counts[space.index[sim.s.tobytes()]] += 1
    e = n / len(space)
    chi2 = ((counts - e) ** 2 / e).sum()
    dof = len(space) - 1
    # mild autocorrelation inflates chi2 slightly; 5 sigma of the chi2 law
    assert chi2 < dof + 5 * np.sqrt(2 * dof), chi2


def test_seq_rs_p_q_zero_is_identity(orc):
    sim = orc.SeqRS(16, 0.0, 0.0, seed=1, stream=0)
    before = sim.s.copy()
    sim.run(10)
    assert np.array_equal(before, sim.s)


def test_seq_rs_conserves(orc):
    sim = orc.SeqRS(64, 1.0, 0.0, seed=1, stream=0)
    for _ in range(20):
        sim.run(1)
        assert orc.check_state(sim.s) == 0
