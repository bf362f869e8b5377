"""Oracle: the background component (an extension of the model: each data
event's density is (1 - f) B e^{-Gamma t} / Nhat + f Gamma_b e^{-Gamma_b t}),
pinned by
  * f = 0: the NLL and gradient of the model without background;
  * f -> 1: the NLL of a pure exponential sample, sum (Gamma_b t - ln Gamma_b);
  * the f derivative against central differences;
  * the maximum-likelihood fraction of a sample mixed from known signal and
    background counts (a missing or misnormalised term biases it)."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

M0 = I.MODEL_SMALL
MB = I.with_background(M0)
GB = MB["g_bkg"]


@pytest.fixture(scope="module")
def sample(orc):
    th0 = I.make_theta(M0, I.draw_coefficients(M0, 101))
    mc = I.phase_space(20_000, 202)
    fn = lambda p, t: orc.event_terms(M0, th0, p, t)
    sig = I.draw_data(fn, 1_500, 203, M0, th0, n_env=50_000, batch=1 << 15)
    bp, bt = I.background_events(500, 204, GB)
    p4 = np.concatenate([sig.p4, bp])
    t = np.concatenate([sig.t, bt])
    return th0, p4, t, mc


def _theta_b(th0, f):
    return np.concatenate([th0, [f]])


def test_zero_fraction_is_the_model_without_background(orc, sample):
    th0, p4, t, mc = sample
    v0, g0 = orc.nll_grad(M0, th0, p4, t, mc)
    v1, g1 = orc.nll_grad(MB, _theta_b(th0, 0.0), p4, t, mc)
    assert abs(v1 - v0) <= 1e-12 * abs(v0)
    assert np.allclose(g1[:-1], g0, rtol=1e-10, atol=1e-10 * np.abs(g0).max())


def test_pure_background_limit(orc, sample):
    th0, p4, t, mc = sample
    f = 1.0 - 1e-12
    v = orc.nll(MB, _theta_b(th0, f), p4, t, mc)
    ref = float(np.sum(GB * t - np.log(GB)))
    assert abs(v - ref) <= 1e-8 * abs(ref)


def test_fraction_derivative(orc, sample):
    th0, p4, t, mc = sample
    th = _theta_b(th0, 0.2)
    _, g = orc.nll_grad(MB, th, p4, t, mc)
    h = 1e-6
    tp, tm = th.copy(), th.copy()
    tp[-1] += h
    tm[-1] -= h
    fd = (orc.nll(MB, tp, p4, t, mc) - orc.nll(MB, tm, p4, t, mc)) / (2 * h)
    assert abs(g[-1] - fd) <= 1e-6 * abs(fd)


def test_fitted_fraction_recovers_the_mixture(orc, sample):
    th0, p4, t, mc = sample
    f_true = 500 / 2000
    fs = np.linspace(0.1, 0.4, 31)
    nll = np.array([orc.nll(MB, _theta_b(th0, f), p4, t, mc) for f in fs])
    k = int(np.argmin(nll))
    assert 0 < k < len(fs) - 1
    a, b, _ = np.polyfit(fs[k - 3:k + 4], nll[k - 3:k + 4], 2)
    f_hat, sigma = -b / (2 * a), 1.0 / np.sqrt(2 * a)
    assert 0.005 < sigma < 0.05
    assert abs(f_hat - f_true) < 4 * sigma, (f_hat, sigma)
