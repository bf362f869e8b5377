"""Oracle: a background component together with a Gaussian decay-time
resolution (both extensions of the model): each data event's density at the
measured time t is (1 - f) R(t) / Nhat + f Gamma_b E(Gamma_b; t), where R is
the resolved signal rate and E(a; t) the exponential e^{-a t'} (t' >= 0)
convolved with the resolution. Pinned by
  * f -> 1: the NLL of a pure background sample, sum -ln(Gamma_b E(Gamma_b;
    t)), with E in closed form (SciPy's erfc / erfcx), so the quadrature of
    the background's convolution is checked against it;
  * f = 0: the NLL and gradient of the resolution model without background;
  * a narrow resolution: the NLL and gradient of the background model
    without resolution;
  * the f derivative against central differences;
  * the maximum-likelihood fraction of a smeared sample mixed from known
    signal and background counts."""

import numpy as np
import pytest
from scipy.special import erfc, erfcx

from paper_1702_06735_amd import inputs as I

M0 = I.MODEL_SMALL
S = 0.06
MB = I.with_background(M0)
MR = I.with_resolution(M0, S)
MBR = I.with_resolution(MB, S)
GB = MB["g_bkg"]


def _E(a, t, s):
    u = (a * s * s - t) / (np.sqrt(2) * s)
    if u >= 0:
        return 0.5 * np.exp(-t * t / (2 * s * s)) * erfcx(u)
    return 0.5 * np.exp(a * a * s * s / 2 - a * t) * erfc(u)


@pytest.fixture(scope="module")
def sample(orc):
    th0 = I.make_theta(M0, I.draw_coefficients(M0, 141), x=0.2, y=0.1)
    mc = I.phase_space(20_000, 242)
    fn = lambda p, t: orc.event_terms(M0, th0, p, t)
    sig = I.draw_data(fn, 1_500, 243, M0, th0, n_env=50_000, batch=1 << 15)
    bp, bt = I.background_events(500, 244, GB)
    p4 = np.concatenate([sig.p4, bp])
    t_true = np.concatenate([sig.t, bt])
    t = t_true + S * np.random.default_rng(245).standard_normal(len(t_true))
    return th0, p4, t_true, t, mc


def _tb(th0, f):
    return np.concatenate([th0, [f]])


def test_pure_background_limit_closed_form(orc, sample):
    th0, p4, _, t, mc = sample
    assert (t < 0).any()
    f = 1.0 - 1e-12
    v = orc.nll(MBR, _tb(th0, f), p4, t, mc)
    ref = -sum(np.log(GB * _E(GB, ti, S)) for ti in t)
    assert abs(v - ref) <= 1e-9 * abs(ref)


def test_zero_fraction_is_the_resolution_model(orc, sample):
    th0, p4, _, t, mc = sample
    v0, g0 = orc.nll_grad(MR, th0, p4, t, mc)
    v1, g1 = orc.nll_grad(MBR, _tb(th0, 0.0), p4, t, mc)
    assert abs(v1 - v0) <= 1e-12 * abs(v0)
    assert np.allclose(g1[:-1], g0, rtol=1e-10, atol=1e-10 * np.abs(g0).max())


def test_narrow_resolution_is_the_background_model(orc, sample):
    th0, p4, t_true, _, mc = sample
    th = _tb(th0, 0.25)
    v0, g0 = orc.nll_grad(MB, th, p4, t_true, mc)
    v1, g1 = orc.nll_grad(I.with_resolution(MB, 1e-7), th, p4, t_true, mc)
    assert abs(v1 - v0) <= 1e-9 * abs(v0)
    assert np.allclose(g1, g0, rtol=1e-6, atol=1e-7 * np.abs(g0).max())


def test_fraction_derivative(orc, sample):
    th0, p4, _, t, mc = sample
    th = _tb(th0, 0.2)
    _, g = orc.nll_grad(MBR, th, p4, t, mc)
    h = 1e-6
    tp, tm = th.copy(), th.copy()
    tp[-1] += h
    tm[-1] -= h
    fd = (orc.nll(MBR, tp, p4, t, mc) - orc.nll(MBR, tm, p4, t, mc)) / (2 * h)
    assert abs(g[-1] - fd) <= 1e-6 * abs(fd)


def test_fitted_fraction_recovers_the_mixture(orc, sample):
    th0, p4, _, t, mc = sample
    f_true = 500 / 2000
    fs = np.linspace(0.1, 0.4, 31)
    nll = np.array([orc.nll(MBR, _tb(th0, f), p4, t, mc) for f in fs])
    k = int(np.argmin(nll))
    assert 0 < k < len(fs) - 1
    a, b, _ = np.polyfit(fs[k - 3:k + 4], nll[k - 3:k + 4], 2)
    f_hat, sigma = -b / (2 * a), 1.0 / np.sqrt(2 * a)
    assert 0.005 < sigma < 0.05
    assert abs(f_hat - f_true) < 4 * sigma, (f_hat, sigma)
