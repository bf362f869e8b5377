"""Oracle: Gaussian decay-time resolution (an extension of Eq. (1)): the
density of the measured time is the rate convolved with the resolution,
integrated by adaptive quadrature. Pinned by
  * x = y = 0: R(t) = 2 |A|^2 E(Gamma; t) with the closed form
    E(a; t) = 1/2 exp(a^2 s^2/2 - a t) erfc((a s^2 - t)/(sqrt 2 s)) (SciPy's
    erfc / erfcx);
  * normalisation: the integral of R over all measured times equals the
    time-integrated rate;
  * a narrow resolution reproduces the NLL without resolution;
  * the x, y derivatives against central differences."""

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import erfc, erfcx

from paper_1702_06735_amd import inputs as I

M0 = I.MODEL_SMALL
S = 0.06


def with_res(model, s=S):
    return dict(model, sigma_t=s)


@pytest.fixture(scope="module")
def sample(orc):
    th0 = I.make_theta(M0, I.draw_coefficients(M0, 101))
    mc = I.phase_space(20_000, 232)
    fn = lambda p, t: orc.event_terms(M0, th0, p, t)
    d = I.draw_data(fn, 1_500, 233, M0, th0, n_env=50_000, batch=1 << 15)
    t = d.t + S * np.random.default_rng(7).standard_normal(len(d.t))
    return th0, d.p4, d.t, t, mc


def _E(a, t, s):
    u = (a * s * s - t) / (np.sqrt(2) * s)
    if u >= 0:
        return 0.5 * np.exp(-t * t / (2 * s * s)) * erfcx(u)
    return 0.5 * np.exp(a * a * s * s / 2 - a * t) * erfc(u)


def test_no_mixing_closed_form(orc, sample):
    th0, p4, _, t, _ = sample
    th = th0.copy()
    th[I.theta_index(M0, "x")] = th[I.theta_index(M0, "y")] = 0.0
    G = 1 / M0["tau"]
    n = 300
    terms = orc.event_terms(with_res(M0), th, p4[:n], t[:n])
    ref = np.array([2 * terms[i, 0] * _E(G, t[i], S) for i in range(n)])
    assert np.allclose(terms[:, 4], ref, rtol=1e-12, atol=0)


def test_normalisation_is_unchanged(orc, sample):
    th0, p4, _, _, _ = sample
    th = th0.copy()
    th[I.theta_index(M0, "x")], th[I.theta_index(M0, "y")] = 0.3, 0.2  # visible mixing
    ev = p4[:1]
    T = orc.event_terms(M0, th, ev)[0, 4]
    f = lambda tt: orc.event_terms(with_res(M0), th, ev, np.array([tt]))[0, 4]
    val = quad(f, -12 * S, 0.0, epsabs=0, epsrel=1e-12, limit=200)[0] + \
        quad(f, 0.0, 60.0, epsabs=0, epsrel=1e-12, limit=400)[0]
    assert abs(val - T) <= 1e-9 * T


def test_narrow_resolution_is_the_model_without_resolution(orc, sample):
    th0, p4, t_true, _, mc = sample
    v0 = orc.nll(M0, th0, p4, t_true, mc)
    v1 = orc.nll(with_res(M0, 1e-7), th0, p4, t_true, mc)
    assert abs(v1 - v0) <= 1e-9 * abs(v0)


def test_xy_derivatives(orc, sample):
    th0, p4, _, t, mc = sample
    m = with_res(M0)
    th = th0.copy()
    th[I.theta_index(M0, "x")], th[I.theta_index(M0, "y")] = 0.3, 0.2
    _, g = orc.nll_grad(m, th, p4, t, mc)
    for name in ("x", "y"):
        j = I.theta_index(M0, name)
        h = 1e-6
        tp, tm = th.copy(), th.copy()
        tp[j] += h
        tm[j] -= h
        fd = (orc.nll(m, tp, p4, t, mc) - orc.nll(m, tm, p4, t, mc)) / (2 * h)
        assert abs(g[j] - fd) <= 1e-6 * abs(fd), (name, g[j], fd)
