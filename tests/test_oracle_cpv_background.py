"""Oracle: CP violation in mixing together with a background component (both
extensions). A tagged data event's density is (1 - f) B_tau e^{-Gamma t} /
Nhat_tau + f Gamma_b e^{-Gamma_b t}: the signal with Abar_f -> (q/p)^tau
Abar_f and its own flavour's normalisation, the background the same for both
flavours. Pinned by
  * f = 0: the NLL and gradient of the model with CP violation alone;
  * q/p = 1: the NLL and gradient of the background model (any tags), with
    zero derivatives in |q/p| and arg(q/p) only if the two flavours balance,
    so those are checked by central differences instead;
  * all tags +1: the background model whose Abar_f coefficients are
    multiplied by q/p;
  * the f, |q/p| and arg(q/p) derivatives against central differences;
  * with a decay-time resolution as well: f = 0 gives CP violation with
    resolution."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

M0 = I.MODEL_SMALL
MB = I.with_background(M0)
MCB = I.with_background(I.with_cp_violation(M0))
GB = MB["g_bkg"]
NC = len(M0["comp_a"]) + len(M0["comp_ab"])


@pytest.fixture(scope="module")
def sample(orc):
    th0 = I.make_theta(M0, I.draw_coefficients(M0, 151))
    mc = I.phase_space(20_000, 252)
    fn = lambda p, t: orc.event_terms(M0, th0, p, t)
    sig = I.draw_data(fn, 1_500, 253, M0, th0, n_env=50_000, batch=1 << 15)
    bp, bt = I.background_events(500, 254, GB)
    p4 = np.concatenate([sig.p4, bp])
    t = np.concatenate([sig.t, bt])
    tags = np.where(np.random.default_rng(255).random(2_000) < 0.5, 1, -1).astype(np.int8)
    return th0, p4, t, tags, mc


def _th(th0, r, phi, f):
    return np.concatenate([th0, [r, phi, f]])


def test_zero_fraction_is_cp_violation_alone(orc, sample):
    th0, p4, t, tags, mc = sample
    mc_only = I.with_cp_violation(M0)
    v0, g0 = orc.nll_tagged(mc_only, np.concatenate([th0, [1.2, 0.4]]), p4, t, tags, mc, grad=True)
    v1, g1 = orc.nll_tagged(MCB, _th(th0, 1.2, 0.4, 0.0), p4, t, tags, mc, grad=True)
    assert abs(v1 - v0) <= 1e-12 * abs(v0)
    assert np.allclose(g1[:-1], g0, rtol=1e-10, atol=1e-10 * np.abs(g0).max())


def test_no_cp_violation_is_the_background_model(orc, sample):
    th0, p4, t, tags, mc = sample
    th_b = np.concatenate([th0, [0.2]])
    v0, g0 = orc.nll_grad(MB, th_b, p4, t, mc)
    v1, g1 = orc.nll_tagged(MCB, _th(th0, 1.0, 0.0, 0.2), p4, t, tags, mc, grad=True)
    assert abs(v1 - v0) <= 1e-12 * abs(v0)
    std = np.r_[np.arange(len(th0)), len(th0) + 2]
    assert np.allclose(g1[std], g0, rtol=1e-10, atol=1e-10 * np.abs(g0).max())


def test_one_flavour_is_the_background_model_with_scaled_abar(orc, sample):
    th0, p4, t, _, mc = sample
    r, phi = 1.3, 0.7
    mu = r * np.exp(1j * phi)
    th = np.array(th0, copy=True)
    na = len(M0["comp_a"])
    c = (th[2 * na:2 * NC:2] + 1j * th[2 * na + 1:2 * NC:2]) * mu
    th[2 * na:2 * NC:2], th[2 * na + 1:2 * NC:2] = c.real, c.imag
    v0 = orc.nll(MB, np.concatenate([th, [0.2]]), p4, t, mc)
    v1 = orc.nll_tagged(MCB, _th(th0, r, phi, 0.2), p4, t, np.ones(len(t), np.int8), mc)
    assert abs(v1 - v0) <= 1e-12 * abs(v0)


@pytest.mark.parametrize("k", [-3, -2, -1])
def test_extra_derivatives(orc, sample, k):
    th0, p4, t, tags, mc = sample
    th = _th(th0, 1.2, 0.4, 0.2)
    _, g = orc.nll_tagged(MCB, th, p4, t, tags, mc, grad=True)
    h = 1e-6
    tp, tm = th.copy(), th.copy()
    tp[k] += h
    tm[k] -= h
    fd = (orc.nll_tagged(MCB, tp, p4, t, tags, mc) - orc.nll_tagged(MCB, tm, p4, t, tags, mc)) / (2 * h)
    assert abs(g[k] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max())


def test_with_resolution_zero_fraction_is_cp_violation_with_resolution(orc, sample):
    th0, p4, t, tags, mc = sample
    ts = t + 0.06 * np.random.default_rng(256).standard_normal(len(t))
    mcr = I.with_resolution(I.with_cp_violation(M0), 0.06)
    mcbr = I.with_resolution(MCB, 0.06)
    v0, g0 = orc.nll_tagged(mcr, np.concatenate([th0, [1.2, 0.4]]), p4, ts, tags, mc, grad=True)
    v1, g1 = orc.nll_tagged(mcbr, _th(th0, 1.2, 0.4, 0.0), p4, ts, tags, mc, grad=True)
    assert abs(v1 - v0) <= 1e-12 * abs(v0)
    assert np.allclose(g1[:-1], g0, rtol=1e-10, atol=1e-10 * np.abs(g0).max())
