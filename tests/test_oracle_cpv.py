"""Oracle: CP violation in mixing (an extension; Eq. (1) assumes none). A
data event with flavour tag tau = +1 (D0) or -1 (D0bar, given as its CP
conjugate) has Eq. (1) with Abar_f -> (q/p)^tau Abar_f, and each flavour its
own normalisation. Pinned by
  * q/p = 1: the NLL and gradient of the model without CP violation, for any
    tags;
  * all tags +1 (or all -1): the model without CP violation whose Abar_f
    coefficients are multiplied by q/p (or by p/q) -- the rate depends on
    Abar_f only through that product;
  * the |q/p| and arg(q/p) derivatives against central differences;
  * a fit of arg(q/p) to tagged samples generated at a known phase."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

M0 = I.MODEL_SMALL
MC_ = I.with_cp_violation(M0)
NC = len(M0["comp_a"]) + len(M0["comp_ab"])


def scale_abar(theta0, mu):
    """theta of the model without CP violation with Abar_f coefficients x mu."""
    th = np.array(theta0, copy=True)
    na = len(M0["comp_a"])
    c = th[2 * na:2 * NC:2] + 1j * th[2 * na + 1:2 * NC:2]
    c = c * mu
    th[2 * na:2 * NC:2] = c.real
    th[2 * na + 1:2 * NC:2] = c.imag
    return th


@pytest.fixture(scope="module")
def sample(orc):
    th0 = I.make_theta(M0, I.draw_coefficients(M0, 101))
    mc = I.phase_space(20_000, 212)
    fn = lambda p, t: orc.event_terms(M0, th0, p, t)
    d = I.draw_data(fn, 2_000, 213, M0, th0, n_env=50_000, batch=1 << 15)
    tags = np.where(np.random.default_rng(5).random(2_000) < 0.5, 1, -1).astype(np.int8)
    return th0, d.p4, d.t, tags, mc


def _cp(th0, r, phi):
    return np.concatenate([th0, [r, phi]])


def test_no_cp_violation_is_the_standard_model(orc, sample):
    th0, p4, t, tags, mc = sample
    v0, g0 = orc.nll_grad(M0, th0, p4, t, mc)
    v1, g1 = orc.nll_tagged(MC_, _cp(th0, 1.0, 0.0), p4, t, tags, mc, grad=True)
    assert abs(v1 - v0) <= 1e-12 * abs(v0)
    assert np.allclose(g1[:-2], g0, rtol=1e-10, atol=1e-10 * np.abs(g0).max())


@pytest.mark.parametrize("tau", [1, -1])
def test_one_flavour_is_the_standard_model_with_scaled_abar(orc, sample, tau):
    th0, p4, t, _, mc = sample
    r, phi = 1.3, 0.7
    mu = (r * np.exp(1j * phi)) ** tau
    tags = np.full(len(t), tau, dtype=np.int8)
    v = orc.nll_tagged(MC_, _cp(th0, r, phi), p4, t, tags, mc)
    ref = orc.nll(M0, scale_abar(th0, mu), p4, t, mc)
    assert abs(v - ref) <= 1e-12 * abs(ref)


def test_qp_derivatives(orc, sample):
    # x, y enlarged so that the q/p dependence is well above the rounding of
    # the difference quotient
    th0, p4, t, tags, mc = sample
    th0 = th0.copy()
    th0[I.theta_index(M0, "x")], th0[I.theta_index(M0, "y")] = 0.3, 0.2
    th = _cp(th0, 1.2, 0.4)
    _, g = orc.nll_tagged(MC_, th, p4, t, tags, mc, grad=True)
    for j in (-2, -1):
        h = 1e-6
        tp, tm = th.copy(), th.copy()
        tp[j] += h
        tm[j] -= h
        fd = (orc.nll_tagged(MC_, tp, p4, t, tags, mc) - orc.nll_tagged(MC_, tm, p4, t, tags, mc)) / (2 * h)
        assert abs(g[j] - fd) <= 1e-6 * max(abs(fd), 1e-3), (j, g[j], fd)


def test_fitted_phase_recovers_the_generated_one(orc):
    """D0 events generated with Abar_f x q/p and D0bar events (as their CP
    conjugates) with Abar_f x p/q, at |q/p| = 1, arg(q/p) = 0.6 and enlarged
    x, y so that the phase is measurable in a small sample."""
    th0 = I.make_theta(M0, I.draw_coefficients(M0, 121), x=0.3, y=0.2)
    r, phi = 1.0, 0.6
    mc = I.phase_space(20_000, 222)
    parts = []
    for tau, seed in ((1, 223), (-1, 224)):
        thp = scale_abar(th0, (r * np.exp(1j * phi)) ** tau)
        fn = lambda p, t, thp=thp: orc.event_terms(M0, thp, p, t)
        d = I.draw_data(fn, 2_000, seed, M0, thp, n_env=50_000, batch=1 << 15)
        parts.append((d.p4, d.t, np.full(len(d.t), tau, dtype=np.int8)))
    p4 = np.concatenate([q[0] for q in parts])
    t = np.concatenate([q[1] for q in parts])
    tags = np.concatenate([q[2] for q in parts])
    phis = np.linspace(0.3, 0.9, 25)
    nll = np.array([orc.nll_tagged(MC_, _cp(th0, r, f), p4, t, tags, mc) for f in phis])
    k = int(np.argmin(nll))
    assert 2 < k < len(phis) - 3
    a, b, _ = np.polyfit(phis[k - 3:k + 4], nll[k - 3:k + 4], 2)
    f_hat, sigma = -b / (2 * a), 1.0 / np.sqrt(2 * a)
    assert sigma < 0.15
    assert abs(f_hat - phi) < 4 * sigma, (f_hat, sigma)
