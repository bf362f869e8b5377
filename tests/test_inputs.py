"""Pins of the seeded input generators (GENBOD phase space, decay times,
accept-reject pseudo-data)."""

import math

import numpy as np
import pytest
from scipy import stats

from paper_1702_06735_amd import inputs as I
from phase_space_checks import constraint_error, isotropy_ok, msq as _msq, pair_mass_pvalue

C = I.MODEL_FULL
MD, MK, MPI = C["m_D"], C["m_K"], C["m_pi"]
MASSES = np.array([MK, MPI, MPI, MPI])


@pytest.fixture(scope="module")
def ev():
    return I.phase_space(200_000, 2024)


def test_four_body_constraints(ev):
    assert constraint_error(ev, MD, MASSES) <= 1e-12


def test_weight_bound_never_exceeded():
    rng = np.random.default_rng(8)
    for _ in range(5):
        r = np.sort(rng.random((1_000_000, 2)), axis=1)
        w, _ = I.genbod_weights(MD, tuple(MASSES), r)
        assert w.max() <= I.genbod_wmax(MD, tuple(MASSES))


def test_pair_mass_density_matches_phase_space(ev):
    """(m(K+ pi-a), m(pi+ pi-b)) is distributed as q(M; m1, m2) q(m1) q(m2)."""
    assert pair_mass_pvalue(ev, MD, MK, MPI) > 1e-4


def test_directions_isotropic(ev):
    assert isotropy_ok(ev)


def test_seed_reproducible():
    a = I.phase_space(1000, 5)
    b = I.phase_space(1000, 5)
    c = I.phase_space(1000, 6)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_decay_time_mixture_mean():
    G, y = 1 / 0.4101, 0.3
    rng = np.random.Generator(np.random.PCG64(9))
    t = I.decay_times(rng, 1_000_000, G, y)
    # mean of exp(-G t) cosh(y G t): (1 + y^2) / (G (1 - y^2))
    mean = (1 + y * y) / (G * (1 - y * y))
    assert abs(t.mean() - mean) < 5 * t.std() / math.sqrt(t.size)


def test_accept_reject_exact_exponential_when_no_mixing():
    """With a rate that is flat in t (x = y = 0) the accepted times must be
    exactly exponential and the phase-space weights must follow the rate."""
    G = 1 / C["tau"]
    th = I.make_theta(C, I.draw_coefficients(C, 3), x=0.0, y=0.0)

    def terms(p4, t):
        # a toy rate depending only on one pair mass: |A|^2 = s(K+ pi-a)
        s = _msq(p4[:, 0] + p4[:, 1])
        out = np.zeros((len(p4), 5))
        out[:, 0] = s
        out[:, 4] = 2 * s
        return out

    d = I.draw_data(terms, 20_000, 17, C, th, n_env=50_000, batch=1 << 15)
    assert d.exceedances == 0
    assert len(d.t) == 20_000
    ks = stats.kstest(d.t, "expon", args=(0, 1 / G))
    assert ks.pvalue > 1e-4
    # accepted events are weighted by s: <s>_accepted = <s^2>/<s> over uniform
    u = I.phase_space(200_000, 18)
    su = _msq(u[:, 0] + u[:, 1])
    sa = _msq(d.p4[:, 0] + d.p4[:, 1])
    ref = (su ** 2).mean() / su.mean()
    assert abs(sa.mean() - ref) < 5 * sa.std() / math.sqrt(sa.size)


def test_accept_reject_restarts_on_exceedance():
    th = I.make_theta(C, I.draw_coefficients(C, 3), x=0.0, y=0.0)

    def terms(p4, t):
        s = _msq(p4[:, 0] + p4[:, 1])
        out = np.zeros((len(p4), 5))
        out[:, 0] = s
        out[:, 4] = 2 * s
        return out

    # a safety factor below 1 is exceeded; the draw must enlarge the envelope
    d = I.draw_data(terms, 2000, 5, C, th, n_env=2000, batch=1 << 14, safety=0.5)
    assert d.exceedances == 0
    u = I.phase_space(200_000, 6)
    assert d.envelope >= _msq(u[:, 0] + u[:, 1]).max()
