"""GPU: CP violation in mixing together with a background component (and
with a decay-time resolution as well), through the C-ABI: NLL and gradient
against the oracle's tagged NLL, and f = 0 against CP violation alone. The
background events are uniform in phase space, tagged at random; those
tagged D0bar go to the library as CP-conjugate records, like the signal's."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I
from test_gpu_cpv import _tagged

pytestmark = pytest.mark.gpu
GB = 1.0 / 0.8


@pytest.fixture(scope="module")
def M():
    from paper_1702_06735_amd import mixamp
    mixamp.load_library()
    return mixamp


@pytest.fixture(scope="module", params=["small", "full"])
def case(request, orc):
    m0 = I.MODEL_SMALL if request.param == "small" else I.MODEL_FULL
    th0 = I.make_theta(m0, I.draw_coefficients(m0, 431), x=0.05, y=0.03)
    mc = I.phase_space(20_011, 432)
    p4, t, tags, p_d0, t_d0, rec_bar, t_bar = _tagged(orc, m0, th0, 1.15, 0.5, (1_201, 1_003), 433)
    bp, bt = I.background_events(600, 434, GB)
    bp = bp.reshape(-1, 16)
    btag = np.where(np.random.default_rng(435).random(600) < 0.5, 1, -1).astype(np.int8)
    p4 = np.concatenate([p4, bp])
    t = np.concatenate([t, bt])
    tags = np.concatenate([tags, btag])
    p_d0 = np.concatenate([p_d0, bp[btag > 0]])
    t_d0 = np.concatenate([t_d0, bt[btag > 0]])
    rec_bar = np.concatenate([rec_bar, I.cp_conjugate(bp[btag < 0]).reshape(-1, 16)])
    t_bar = np.concatenate([t_bar, bt[btag < 0]])
    model = I.with_background(I.with_cp_violation(m0), GB)
    return m0, model, th0, mc, (p4, t, tags, p_d0, t_d0, rec_bar, t_bar)


def _ctx(M, model, mc, smp, t_d0=None, t_bar=None):
    _, _, _, p_d0, td0, rec_bar, tbar = smp
    c = M.Context(model, device=0)
    c.load_events(M.MXA_MC, mc)
    c.load_events(M.MXA_DATA, p_d0, td0 if t_d0 is None else t_d0)
    c.load_events(M.MXA_DATA_BAR, rec_bar, tbar if t_bar is None else t_bar)
    return c


def test_nll_and_gradient_match_the_oracle(orc, M, case):
    m0, model, th0, mc, smp = case
    p4, t, tags = smp[:3]
    th = np.concatenate([th0, [1.15, 0.5, 0.2]])
    ref, _, _, S = orc.nll_tagged(model, th, p4, t, tags, mc, diag=True)
    ref_g = orc.nll_tagged(model, th, p4, t, tags, mc, grad=True)[1]
    with _ctx(M, model, mc, smp) as c:
        c.set_params(th)
        v64, g64 = c.nll_grad("fp64")
        n64 = c.nll("fp64")
        v32, g32 = c.nll_grad("fp32amp")
    assert abs(v64 - ref) <= 1e-12 * abs(ref) and abs(n64 - ref) <= 1e-12 * abs(ref)
    assert np.abs(g64 - ref_g).max() <= 1e-9 * np.abs(ref_g).max()
    assert abs(v32 - ref) <= 1e-6 * S
    assert np.abs(g32 - ref_g).max() <= 1e-3 * np.abs(ref_g).max()


def test_with_resolution_matches_the_oracle(orc, M, case):
    m0, model, th0, mc, smp = case
    p4, t, tags, _, t_d0, _, t_bar = smp
    rng = np.random.default_rng(436)
    sm_d0 = t_d0 + 0.06 * rng.standard_normal(len(t_d0))
    sm_bar = t_bar + 0.06 * rng.standard_normal(len(t_bar))
    # the oracle's view: D0-tagged events first, then the D0bar ones, in the
    # order the fixture built them
    n_sig_d0 = int(np.sum(tags[:len(tags) - 600] > 0))
    n_sig_bar = len(tags) - 600 - n_sig_d0
    btag = tags[len(tags) - 600:]
    ts = np.concatenate([sm_d0[:n_sig_d0], sm_bar[:n_sig_bar], np.empty(600)])
    ts[len(tags) - 600:][btag > 0] = sm_d0[n_sig_d0:]
    ts[len(tags) - 600:][btag < 0] = sm_bar[n_sig_bar:]
    mr = I.with_resolution(model, 0.06)
    th = np.concatenate([th0, [1.15, 0.5, 0.2]])
    ref = orc.nll_tagged(mr, th, p4, ts, tags, mc)
    ref_g = orc.nll_tagged(mr, th, p4, ts, tags, mc, grad=True)[1]
    with _ctx(M, mr, mc, smp, sm_d0, sm_bar) as c:
        c.set_params(th)
        v, g = c.nll_grad("fp64")
    assert abs(v - ref) <= 1e-12 * abs(ref)
    assert np.abs(g - ref_g).max() <= 1e-9 * np.abs(ref_g).max()


def test_zero_fraction_equals_cp_violation_alone(M, case):
    m0, model, th0, mc, smp = case
    with _ctx(M, I.with_cp_violation(m0), mc, smp) as c:
        c.set_params(np.concatenate([th0, [1.15, 0.5]]))
        v0, g0 = c.nll_grad("fp64")
    with _ctx(M, model, mc, smp) as c:
        c.set_params(np.concatenate([th0, [1.15, 0.5, 0.0]]))
        v1, g1 = c.nll_grad("fp64")
    assert abs(v1 - v0) <= 1e-12 * abs(v0)
    assert np.abs(g1[:-1] - g0).max() <= 1e-9 * np.abs(g0).max()
