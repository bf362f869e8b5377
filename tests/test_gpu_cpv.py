"""GPU: CP violation in mixing (q/p = |q/p| e^{i phi} free; D0-tagged data in
MXA_DATA, D0bar-tagged data in MXA_DATA_BAR as D0bar records, which the
library takes to their CP conjugates), through the C-ABI: NLL and gradient
against the oracle's tagged NLL (which implements the per-event
(q/p)^tau Abar_f and the per-flavour normalisation from the definition), q/p
= 1 against the model without CP violation, refusals, and a fit of the phase
to samples generated at a known one."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    from paper_1702_06735_amd import mixamp
    mixamp.load_library()
    return mixamp


def scale_abar(model, theta0, mu):
    th = np.array(theta0, copy=True)
    na, nc = len(model["comp_a"]), len(model["comp_a"]) + len(model["comp_ab"])
    c = (th[2 * na:2 * nc:2] + 1j * th[2 * na + 1:2 * nc:2]) * mu
    th[2 * na:2 * nc:2], th[2 * na + 1:2 * nc:2] = c.real, c.imag
    return th


def _tagged(orc, m0, th0, r, phi, n_each, seed):
    """D0 events at Abar x q/p and D0bar events (generated as their CP
    conjugates at Abar x p/q); returns the oracle's view (D0-frame events and
    tags) and the D0bar records for the library."""
    parts = []
    for tau, sd in ((1, seed), (-1, seed + 1)):
        thp = scale_abar(m0, th0, (r * np.exp(1j * phi)) ** tau)
        fn = lambda p, t, thp=thp: orc.event_terms(m0, thp, p, t)
        d = I.draw_data(fn, n_each[0 if tau > 0 else 1], sd, m0, thp, n_env=60_000, batch=1 << 15)
        parts.append((d.p4.reshape(-1, 16), d.t))
    (p_d0, t_d0), (p_bar, t_bar) = parts
    tags = np.concatenate([np.ones(len(t_d0)), -np.ones(len(t_bar))]).astype(np.int8)
    return (np.concatenate([p_d0, p_bar]), np.concatenate([t_d0, t_bar]), tags,
            p_d0, t_d0, I.cp_conjugate(p_bar).reshape(-1, 16), t_bar)


@pytest.fixture(scope="module", params=["small", "full"])
def case(request, orc):
    m0 = I.MODEL_SMALL if request.param == "small" else I.MODEL_FULL
    th0 = I.make_theta(m0, I.draw_coefficients(m0, 331), x=0.05, y=0.03)
    mc = I.phase_space(20_011, 332)
    smp = _tagged(orc, m0, th0, 1.15, 0.5, (1_501, 1_203), 333)
    return m0, I.with_cp_violation(m0), th0, mc, smp


def _ctx(M, model, mc, smp):
    _, _, _, p_d0, t_d0, rec_bar, t_bar = smp
    c = M.Context(model, device=0)
    c.load_events(M.MXA_MC, mc)
    c.load_events(M.MXA_DATA, p_d0, t_d0)
    c.load_events(M.MXA_DATA_BAR, rec_bar, t_bar)
    return c


def test_nll_and_gradient_match_the_oracle(orc, M, case):
    m0, mc_model, th0, mc, smp = case
    p4, t, tags = smp[:3]
    th = np.concatenate([th0, [1.15, 0.5]])
    ref, _, _, S = orc.nll_tagged(mc_model, th, p4, t, tags, mc, diag=True)
    ref_g = orc.nll_tagged(mc_model, th, p4, t, tags, mc, grad=True)[1]
    with _ctx(M, mc_model, mc, smp) as c:
        c.set_params(th)
        v64, g64 = c.nll_grad("fp64")
        n64 = c.nll("fp64")
        v32, g32 = c.nll_grad("fp32amp")
    assert abs(v64 - ref) <= 1e-12 * abs(ref) and abs(n64 - ref) <= 1e-12 * abs(ref)
    assert np.abs(g64 - ref_g).max() <= 1e-9 * np.abs(ref_g).max()
    assert abs(v32 - ref) <= 1e-6 * S
    assert np.abs(g32 - ref_g).max() <= 1e-3 * np.abs(ref_g).max()


def test_no_cp_violation_equals_the_standard_model(M, case):
    m0, mc_model, th0, mc, smp = case
    p4, t = smp[0], smp[1]
    with M.Context(m0, device=0) as c:
        c.load_events(M.MXA_MC, mc)
        c.load_events(M.MXA_DATA, p4, t)
        c.set_params(th0)
        v0, g0 = c.nll_grad("fp64")
    with _ctx(M, mc_model, mc, smp) as c:
        c.set_params(np.concatenate([th0, [1.0, 0.0]]))
        v1, g1 = c.nll_grad("fp64")
    assert abs(v1 - v0) <= 1e-12 * abs(v0)
    assert np.abs(g1[:-2] - g0).max() <= 1e-9 * np.abs(g0).max()


def test_refusals(M, case):
    m0, mc_model, th0, mc, smp = case
    th = np.concatenate([th0, [1.1, 0.2]])
    with _ctx(M, mc_model, mc, smp) as c:
        c.set_params(th)
        for call in (lambda: c.nll_multi(th[None, :]),
                     lambda: c.generate(M.MXA_DATA, 10, 1, envelope=1.0)):
            with pytest.raises(M.MixampError) as e:
                call()
            assert e.value.code == M.MXA_EINVAL
        bad = th.copy()
        bad[-2] = 0.0
        with pytest.raises(M.MixampError) as e:
            c.set_params(bad)
        assert e.value.code == M.MXA_EDOMAIN
    with M.Context(m0, device=0) as c:
        with pytest.raises(M.MixampError) as e:
            c.load_events(M.MXA_DATA_BAR, smp[5], smp[6])
        assert e.value.code == M.MXA_EINVAL
    shape = [m0[k] for k in ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1")]
    with pytest.raises(M.MixampError) as e:
        M.Server(mc_model, mc, shape, precision="fp64", max_slots=2)
    assert e.value.code == M.MXA_EINVAL


def test_fit_recovers_the_phase(orc, M):
    m0 = I.MODEL_SMALL
    mc_model = I.with_cp_violation(m0)
    th0 = I.make_theta(m0, I.draw_coefficients(m0, 121), x=0.3, y=0.2)
    mc = I.phase_space(20_000, 342)
    smp = _tagged(orc, m0, th0, 1.0, 0.6, (2_000, 2_000), 343)
    sc = np.zeros(I.n_theta(mc_model))
    sc[-2] = sc[-1] = 0.05
    with _ctx(M, mc_model, mc, smp) as c:
        r = c.fit(np.concatenate([th0, [1.0, 0.0]]), sc, precision="fp64", gtol=1e-6, errors=True)
    assert r["status"] == "converged" and r["errors_ok"], r
    phi, sphi = r["theta"][-1], r["err"][-1]
    rr, sr = r["theta"][-2], r["err"][-2]
    assert sphi < 0.15 and sr < 0.15
    assert abs(phi - 0.6) < 4 * sphi, (phi, sphi)
    assert abs(rr - 1.0) < 4 * sr, (rr, sr)


def test_cp_violation_with_resolution_matches_the_oracle(orc, M):
    """The two extensions together: tagged samples with smeared decay times."""
    m0 = I.MODEL_SMALL
    th0 = I.make_theta(m0, I.draw_coefficients(m0, 371), x=0.1, y=0.05)
    mc = I.phase_space(10_007, 372)
    p4, t, tags, p_d0, t_d0, rec_bar, t_bar = _tagged(orc, m0, th0, 0.9, -0.4, (1_001, 803), 373)
    rng = np.random.default_rng(374)
    t = t + 0.05 * rng.standard_normal(len(t))
    t_d0, t_bar = t[:len(t_d0)], t[len(t_d0):]
    model = dict(I.with_cp_violation(m0), sigma_t=0.05)
    th = np.concatenate([th0, [0.9, -0.4]])
    ref = orc.nll_tagged(model, th, p4, t, tags, mc)
    ref_g = orc.nll_tagged(model, th, p4, t, tags, mc, grad=True)[1]
    with M.Context(model, device=0) as c:
        c.load_events(M.MXA_MC, mc)
        c.load_events(M.MXA_DATA, p_d0, t_d0)
        c.load_events(M.MXA_DATA_BAR, rec_bar, t_bar)
        c.set_params(th)
        v, g = c.nll_grad("fp64")
    assert abs(v - ref) <= 1e-12 * abs(ref)
    assert np.abs(g - ref_g).max() <= 1e-9 * np.abs(ref_g).max()


@pytest.mark.parametrize("which", ["d0_only", "d0bar_only"])
def test_one_flavour_loaded(orc, M, case, which):
    """With one flavour's sample empty the other alone is evaluated (and the
    empty one adds nothing)."""
    m0, mc_model, th0, mc, smp = case
    p4, t, tags, p_d0, t_d0, rec_bar, t_bar = smp
    th = np.concatenate([th0, [1.15, 0.5]])
    keep = tags > 0 if which == "d0_only" else tags < 0
    ref = orc.nll_tagged(mc_model, th, p4[keep], t[keep], tags[keep], mc)
    with M.Context(mc_model, device=0) as c:
        c.load_events(M.MXA_MC, mc)
        if which == "d0_only":
            c.load_events(M.MXA_DATA, p_d0, t_d0)
        else:
            c.load_events(M.MXA_DATA_BAR, rec_bar, t_bar)
        c.set_params(th)
        v = c.nll("fp64")
    assert abs(v - ref) <= 1e-12 * abs(ref)
