"""GPU: many parameter sets sharing the lineshapes (mxa_nll_multi) against the
oracle's NLL at each set, through the C-ABI."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    from paper_1702_06735_amd import mixamp
    mixamp.load_library()
    return mixamp


@pytest.fixture(scope="module", params=["small", "full"])
def setup(request, orc):
    model = I.MODEL_SMALL if request.param == "small" else I.MODEL_FULL
    th = I.make_theta(model, I.draw_coefficients(model, 301))
    mc = I.phase_space(30_000, 302)
    fn = lambda p, t: orc.event_terms(model, th, p, t)
    d = I.draw_data(fn, 3_001, 303, model, th, n_env=50_000, batch=1 << 16)
    rng = np.random.default_rng(304)
    n_sets = 37                                   # three chunks of 16, the last ragged
    sets = np.repeat(th[None, :], n_sets, axis=0)
    nc = 2 * (len(model["comp_a"]) + len(model["comp_ab"]))
    sets[1:, :nc] += rng.normal(0, 0.05, (n_sets - 1, nc))
    sets[1:, I.theta_index(model, "x")] += rng.uniform(-0.01, 0.01, n_sets - 1)
    sets[1:, I.theta_index(model, "y")] += rng.uniform(-0.01, 0.01, n_sets - 1)
    return model, sets, d.p4, d.t, mc


def test_fp64_sets_match_oracle(orc, M, setup):
    model, sets, pd, td, mc = setup
    with M.Context(model) as ctx:
        ctx.load_events(M.MXA_MC, mc)
        ctx.load_events(M.MXA_DATA, pd, td)
        got = ctx.nll_multi(sets, "fp64")
    for s, th in enumerate(sets):
        ref, _, _, S = orc.nll(model, th, pd, td, mc, diag=True)
        assert abs(got[s] - ref) <= 1e-12 * max(abs(ref), 1e-3 * S), s


def test_fp32amp_sets_within_bound(orc, M, setup):
    model, sets, pd, td, mc = setup
    with M.Context(model) as ctx:
        ctx.load_events(M.MXA_MC, mc)
        ctx.load_events(M.MXA_DATA, pd, td)
        got = ctx.nll_multi(sets, "fp32amp")
        # the same sets one at a time in Gram mode, FP32 amplitudes
        ctx.set_mc_mode(M.MXA_MC_GRAM)
        one = []
        for th in sets[:5]:
            ctx.set_params(th)
            one.append(ctx.nll("fp32amp"))
    for s, th in enumerate(sets):
        ref, _, _, S = orc.nll(model, th, pd, td, mc, diag=True)
        assert abs(got[s] - ref) <= 1e-6 * S, s
    _, _, _, S = orc.nll(model, sets[0], pd, td, mc, diag=True)
    assert np.all(np.abs(got[:5] - np.array(one)) <= 1e-6 * S)


def test_sets_out_of_domain_and_errors(orc, M, setup):
    model, sets, pd, td, mc = setup
    th = sets[:3].copy()
    th[1, I.theta_index(model, "y")] = 1.5
    with M.Context(model) as ctx:
        ctx.load_events(M.MXA_MC, mc)
        ctx.load_events(M.MXA_DATA, pd, td)
        got = ctx.nll_multi(th, "fp64")
        assert np.isinf(got[1]) and np.isfinite(got[0]) and np.isfinite(got[2])
        assert abs(got[2] - orc.nll(model, th[2], pd, td, mc)) <= 1e-12 * abs(got[2])
        bad = sets[:2].copy()
        bad[1, -1] += 0.01                         # another a1 width
        with pytest.raises(M.MixampError) as e:
            ctx.nll_multi(bad)
        assert e.value.code == M.MXA_EINVAL
        with pytest.raises(M.MixampError) as e:
            ctx.nll_multi(np.repeat(sets[:1], 65, axis=0))
        assert e.value.code == M.MXA_EINVAL
        full = ctx.nll_multi(np.repeat(sets[:1], 64, axis=0))
        assert np.all(full == full[0])
        assert abs(full[0] - orc.nll(model, sets[0], pd, td, mc)) <= 1e-12 * abs(full[0])


def test_no_data_gives_zero(M, setup):
    model, sets, pd, td, mc = setup
    with M.Context(model) as ctx:
        ctx.load_events(M.MXA_MC, mc)
        assert np.all(ctx.nll_multi(sets[:4]) == 0.0)
