"""Pins of the oracle's pseudo-experiment generator (Sec. 3.1): Philox4x32-10
random numbers, GENBOD phase space, accept-reject by Eq. (1) with decay
times. The generator is checked against published known answers, the
phase-space density, closed-form time moments and an independent sample
(the fixture generator) reweighted by the oracle's own rate."""

import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1702_06735_amd import inputs as I
from phase_space_checks import constraint_error, isotropy_ok, msq, pair_mass_pvalue

C = I.MODEL_FULL
MD, MK, MPI = C["m_D"], C["m_K"], C["m_pi"]
MASSES = (MK, MPI, MPI, MPI)
WMAX = I.genbod_wmax(MD, MASSES)
G = 1.0 / C["tau"]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(v, 16) for v in r]
        assert oracle.philox(w[0:4], w[4:6]) == w[6:10]


def test_candidate_uniforms_layout():
    """Uniform 2j, 2j+1 of candidate i come from counter (i lo, i hi, j, stream)
    under key (seed lo, seed hi): the top 52 bits of (w0 w1) and (w2 w3)."""
    seed, i, stream = 0x1234_5678_9ABC_DEF0, (7 << 32) | 11, 1
    u = oracle.candidate_uniforms(seed, i, stream)
    for j in range(6):
        w = oracle.philox([i & 0xFFFFFFFF, i >> 32, j, stream],
                          [seed & 0xFFFFFFFF, seed >> 32])
        for h, (a, b) in enumerate(((w[0], w[1]), (w[2], w[3]))):
            k = ((a << 32) | b) >> 12
            assert u[2 * j + h] == (k + 0.5) / 2.0 ** 52
    assert not np.array_equal(u, oracle.candidate_uniforms(seed, i, 0))
    assert not np.array_equal(u, oracle.candidate_uniforms(seed + 1, i, stream))


def test_uniform_moments():
    u = np.array([oracle.candidate_uniforms(99, i, 0) for i in range(20_000)])
    assert u.min() > 0.0 and u.max() < 1.0
    n = u.size
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * math.sqrt(1 / 180 / n)
    # neighbouring uniforms are uncorrelated
    r = np.corrcoef(u[:, :-1].ravel(), u[:, 1:].ravel())[0, 1]
    assert abs(r) < 5 / math.sqrt(n)


@pytest.fixture(scope="module")
def ps():
    return oracle.generate(C, None, "mc", seed=4242, n_cand=400_000, wmax=WMAX)


def test_phase_space_events_are_physical(ps):
    idx, p4, t, st = ps
    assert t is None
    assert st[0] == st[1] == len(idx) and st[2] == 0
    assert constraint_error(p4, MD, MASSES) <= 1e-12
    assert np.all(np.diff(idx) > 0)


def test_phase_space_density_and_isotropy(ps):
    _, p4, _, _ = ps
    assert pair_mass_pvalue(p4, MD, MK, MPI) > 1e-4
    for k in range(4):
        assert isotropy_ok(p4, k)


def test_genbod_acceptance_is_mean_weight_over_bound(ps):
    """Kept fraction = E[w] / wmax, E[w] from the fixture generator's weight
    over sorted uniform pairs."""
    idx, _, _, st = ps
    rng = np.random.default_rng(5)
    w, _ = I.genbod_weights(MD, MASSES, np.sort(rng.random((2_000_000, 2)), axis=1))
    p = w.mean() / WMAX
    n = 400_000
    assert abs(st[1] / n - p) < 5 * math.sqrt(p * (1 - p) / n) + 5 * w.std() / WMAX / math.sqrt(w.size)


def test_candidates_are_independent_of_the_split():
    a = oracle.generate(C, None, "mc", seed=7, n_cand=5000, wmax=WMAX)
    b1 = oracle.generate(C, None, "mc", seed=7, n_cand=2000, wmax=WMAX)
    b2 = oracle.generate(C, None, "mc", seed=7, n_cand=3000, wmax=WMAX, first=2000)
    assert np.array_equal(a[0], np.concatenate([b1[0], b2[0]]))
    assert np.array_equal(a[1], np.concatenate([b1[1], b2[1]]))
    # max_out truncates the output, not the statistics
    c = oracle.generate(C, None, "mc", seed=7, n_cand=5000, wmax=WMAX, max_out=10)
    assert np.array_equal(c[0], a[0][:10]) and c[3] == a[3]


def _envelope(th, n=200_000, seed=31):
    u = I.phase_space(n, seed)
    e = oracle.event_terms(C, th, u)
    return 1.2 * (e[:, 0] + e[:, 1]).max()


def test_data_without_mixing_follows_the_rate():
    """x = y = 0: B = 2|A|^2, so t is exactly exponential and the kept events
    are phase space weighted by |A|^2 (checked against a fixture sample
    reweighted by the oracle's |A|^2)."""
    th = I.make_theta(C, I.draw_coefficients(C, 3), x=0.0, y=0.0)
    env = _envelope(th)
    idx, p4, t, st = oracle.generate(C, th, "data", seed=11, n_cand=4_000_000, wmax=WMAX,
                                     envelope=env)
    assert st[2] == 0 and st[0] == len(t) > 5000
    assert constraint_error(p4, MD, MASSES) <= 1e-12
    assert stats.kstest(t, "expon", args=(0, 1 / G)).pvalue > 1e-4
    u = I.phase_space(300_000, 32)
    w = oracle.event_terms(C, th, u)[:, 0]
    for f in (lambda q: msq(q[:, 0] + q[:, 1]), lambda q: msq(q[:, 2] + q[:, 3]),
              lambda q: msq(q[:, 1] + q[:, 2] + q[:, 3])):
        fd, fu = f(p4), f(u)
        ref = (fu * w).sum() / w.sum()
        # error of the data mean and of the weighted reference
        err = fd.std() / math.sqrt(fd.size) + math.sqrt(((fu - ref) ** 2 * w ** 2).sum()) / w.sum()
        assert abs(fd.mean() - ref) < 5 * err


def test_data_time_moments_with_mixing():
    """With mixing, E[t] of the kept events follows from the phase-space means
    of |A|^2 + |Abar|^2, |A|^2 - |Abar|^2, Re and Im of A Abar* and the closed
    forms of int t e^{-Gt} {cosh, sinh}(yGt) and {cos, sin}(xGt) dt."""
    x, y = 0.35, 0.25
    th = I.make_theta(C, I.draw_coefficients(C, 4), x=x, y=y)
    env = _envelope(th)
    _, _, t, st = oracle.generate(C, th, "data", seed=12, n_cand=4_000_000, wmax=WMAX,
                                  envelope=env)
    assert st[2] == 0
    u = I.phase_space(300_000, 33)
    e = oracle.event_terms(C, th, u)
    S, D, R, Im = (e[:, 0] + e[:, 1]).mean(), (e[:, 0] - e[:, 1]).mean(), e[:, 2].mean(), e[:, 3].mean()
    # zeroth and first time moments of each term
    c0, s0 = 1 / (G * (1 - y * y)), y / (G * (1 - y * y))
    k0, n0 = 1 / (G * (1 + x * x)), x / (G * (1 + x * x))
    c1, s1 = (1 + y * y) / (G * G * (1 - y * y) ** 2), 2 * y / (G * G * (1 - y * y) ** 2)
    k1, n1 = (1 - x * x) / (G * G * (1 + x * x) ** 2), 2 * x / (G * G * (1 + x * x) ** 2)
    m0 = S * c0 + D * k0 - 2 * R * s0 - 2 * Im * n0
    m1 = S * c1 + D * k1 - 2 * R * s1 - 2 * Im * n1
    ref = m1 / m0
    # the phase-space means carry their own sampling error; bound it by the
    # spread of the per-event mean time
    per = (e[:, 0] + e[:, 1]) * c1 + (e[:, 0] - e[:, 1]) * k1 - 2 * e[:, 2] * s1 - 2 * e[:, 3] * n1
    err = t.std() / math.sqrt(t.size) + per.std() / math.sqrt(per.size) / m0 * 2
    assert abs(t.mean() - ref) < 5 * err
    # and the mixing terms matter at this precision
    assert abs(ref - (S * c1 + D * k1) / (S * c0 + D * k0)) > 3 * err


def test_exceedances_are_counted():
    th = I.make_theta(C, I.draw_coefficients(C, 3), x=0.0, y=0.0)
    env = _envelope(th) / 200.0
    _, _, _, st = oracle.generate(C, th, "data", seed=11, n_cand=50_000, wmax=WMAX, envelope=env)
    assert st[2] > 0


def test_invalid_arguments():
    th = I.make_theta(C, I.draw_coefficients(C, 3))
    with pytest.raises(oracle.OracleError):
        oracle.generate(C, th, "data", seed=1, n_cand=10, wmax=WMAX, envelope=0.0)
    with pytest.raises(oracle.OracleError):
        oracle.generate(C, th, "mc", seed=1, n_cand=10, wmax=0.0)
    bad = th.copy()
    bad[I.theta_index(C, "y")] = 1.0
    with pytest.raises(oracle.OracleError):
        oracle.generate(C, bad, "data", seed=1, n_cand=10, wmax=WMAX, envelope=1.0)
