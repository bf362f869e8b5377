"""GPU: models with a background component (each data event's density
(1 - f) B e^{-Gamma t} / Nhat + f Gamma_b e^{-Gamma_b t}), through the
C-ABI: NLL and gradient against the oracle in both precisions, f = 0 against
the model without background, the modes that refuse such models, a fit of
the fraction on a sample mixed from known signal and background counts, and
the same fit on the fit server."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    from paper_1702_06735_amd import mixamp
    mixamp.load_library()
    return mixamp


def _mixed(orc, model0, seed, n_sig, n_bkg, n_mc):
    th0 = I.make_theta(model0, I.draw_coefficients(model0, seed))
    mc = I.phase_space(n_mc, seed + 1)
    fn = lambda p, t: orc.event_terms(model0, th0, p, t)
    sig = I.draw_data(fn, n_sig, seed + 2, model0, th0, n_env=60_000, batch=1 << 15)
    bp, bt = I.background_events(n_bkg, seed + 3, 1.0 / 0.8)
    rng = np.random.default_rng(seed + 4)
    order = rng.permutation(n_sig + n_bkg)
    p4 = np.concatenate([sig.p4.reshape(-1, 16), bp.reshape(-1, 16)])[order]
    t = np.concatenate([sig.t, bt])[order]
    return th0, p4, t, mc


@pytest.fixture(scope="module", params=["small", "full"])
def case(request, orc):
    m0 = I.MODEL_SMALL if request.param == "small" else I.MODEL_FULL
    th0, p4, t, mc = _mixed(orc, m0, 301 if request.param == "small" else 311, 2_251, 750, 20_011)
    return m0, I.with_background(m0), th0, p4, t, mc


def _ctx(M, model, p4, t, mc):
    c = M.Context(model, device=0)
    c.load_events(M.MXA_MC, mc)
    c.load_events(M.MXA_DATA, p4, t)
    return c


def test_nll_and_gradient_match_the_oracle(orc, M, case):
    m0, mb, th0, p4, t, mc = case
    th = np.concatenate([th0, [0.23]])
    ref, _, _, S = orc.nll(mb, th, p4, t, mc, diag=True)
    ref_g = orc.nll_grad(mb, th, p4, t, mc)[1]
    with _ctx(M, mb, p4, t, mc) as c:
        c.set_params(th)
        v64, g64 = c.nll_grad("fp64")
        n64 = c.nll("fp64")
        v32, g32 = c.nll_grad("fp32amp")
        n32 = c.nll("fp32amp")
    assert abs(v64 - ref) <= 1e-12 * abs(ref) and abs(n64 - ref) <= 1e-12 * abs(ref)
    assert np.abs(g64 - ref_g).max() <= 1e-9 * np.abs(ref_g).max()
    assert abs(v32 - ref) <= 1e-6 * S and abs(n32 - ref) <= 1e-6 * S
    assert np.abs(g32 - ref_g).max() <= 1e-3 * np.abs(ref_g).max()


def test_zero_fraction_equals_the_model_without_background(M, case):
    m0, mb, th0, p4, t, mc = case
    with _ctx(M, m0, p4, t, mc) as c:
        c.set_params(th0)
        v0, g0 = c.nll_grad("fp64")
    with _ctx(M, mb, p4, t, mc) as c:
        c.set_params(np.concatenate([th0, [0.0]]))
        v1, g1 = c.nll_grad("fp64")
    assert abs(v1 - v0) <= 1e-12 * abs(v0)
    assert np.abs(g1[:-1] - g0).max() <= 1e-9 * np.abs(g0).max()


def test_gram_mode_equals_the_direct_mc_pass(M, case):
    """In Gram mode the data pass takes Nhat formed on the host from the Gram
    matrix; NLL and gradient equal the direct MC pass's (the masses' and
    widths' entries have no Gram form and are NaN)."""
    m0, mb, th0, p4, t, mc = case
    th = np.concatenate([th0, [0.23]])
    with _ctx(M, mb, p4, t, mc) as c:
        c.set_params(th)
        v_dir, g_dir, d_dir = c.nll_grad("fp64", diag=True)
        n_dir = c.nll("fp64")
        c.set_mc_mode(M.MXA_MC_GRAM)
        v_gr, g_gr = c.nll_grad("fp64")
        n_gr = c.nll("fp64")
        v32, g32 = c.nll_grad("fp32amp")
    S = d_dir[2]
    assert abs(v_gr - v_dir) <= 1e-12 * max(abs(v_dir), 1e-3 * S)
    assert abs(n_gr - n_dir) <= 1e-12 * max(abs(n_dir), 1e-3 * S)
    n_free = 2 * (len(m0["comp_a"]) + len(m0["comp_ab"])) + 2
    keep = np.r_[np.arange(n_free), len(th) - 1]
    gmax = np.abs(g_dir[keep]).max()
    assert np.abs(g_gr[keep] - g_dir[keep]).max() <= 1e-9 * gmax
    assert np.all(np.isnan(g_gr[n_free:len(th) - 1]))
    assert abs(v32 - v_dir) <= 1e-6 * S
    assert np.abs(g32[keep] - g_dir[keep]).max() <= 1e-3 * gmax


@pytest.mark.parametrize("prec", ["fp64", "fp32amp"])
def test_many_sets_equal_single_evaluations(M, case, prec):
    """mxa_nll_multi: sets differing in the coefficients, x, y and the
    fraction, each with its own Nhat from the Gram matrix, against one Gram
    mode evaluation per set; a set outside the domain gives +inf."""
    m0, mb, th0, p4, t, mc = case
    rng = np.random.default_rng(17)
    sets = np.tile(np.concatenate([th0, [0.2]]), (19, 1))
    nc = 2 * (len(m0["comp_a"]) + len(m0["comp_ab"]))
    sets[:, :nc] += rng.normal(0, 0.05, (19, nc))
    sets[:, I.theta_index(mb, "x")] += rng.normal(0, 0.01, 19)
    sets[:, I.theta_index(mb, "y")] += rng.normal(0, 0.01, 19)
    sets[:, -1] = rng.uniform(0.05, 0.5, 19)
    sets[7, -1] = 1.0  # outside the domain
    with _ctx(M, mb, p4, t, mc) as c:
        c.set_mc_mode(M.MXA_MC_GRAM)
        multi = c.nll_multi(sets, prec)
        single = []
        for s in sets:
            if s[-1] >= 1.0:
                single.append(np.inf)
                continue
            c.set_params(s)
            single.append(c.nll(prec))
        c.set_params(sets[0])
        S = c.nll("fp64", diag=True)[1][2]
    single = np.array(single)
    assert np.isinf(multi[7])
    fin = np.isfinite(single)
    # FP32 amplitudes: A_f, Abar_f from the matrix-core product here, from
    # fused multiply-adds in the single evaluation
    tol = 1e-12 * np.abs(single[fin]) if prec == "fp64" else 1e-6 * S
    assert np.all(np.abs(multi[fin] - single[fin]) <= tol)


def test_modes_that_refuse_a_background_component(M, case):
    m0, mb, th0, p4, t, mc = case
    th = np.concatenate([th0, [0.1]])
    with _ctx(M, mb, p4, t, mc) as c:
        c.set_params(th)
        # a fraction outside [0, 1) is outside the domain
        bad = th.copy()
        bad[-1] = 1.0
        with pytest.raises(M.MixampError) as e:
            c.set_params(bad)
        assert e.value.code == M.MXA_EDOMAIN
    # the streamed server (lineshapes floating) has no Nhat before its data
    # pass: it refuses the model
    with pytest.raises(M.MixampError) as e:
        M.Server(mb, mc, None, precision="fp64", max_slots=2)
    assert e.value.code == M.MXA_EINVAL


@pytest.mark.parametrize("prec", ["fp64", "fp32amp"])
def test_server_fit_equals_the_context_fit(orc, M, case, prec):
    """The fit server (the MC through its Gram matrix; each tick forms every
    fit's Nhat before the data pass) against mxa_fit on a context (the MC
    summed event by event): one likelihood, so one fitted point, to 1% of the
    errors; in FP64 the server's NLL and gradient there are the oracle's."""
    m0, mb, th0, p4, t, mc = case
    sc = np.zeros(I.n_theta(mb))
    sc[I.theta_index(mb, "x")] = sc[I.theta_index(mb, "y")] = 1e-3
    sc[-1] = 0.05
    free = sc > 0
    start = np.concatenate([th0, [0.1]])
    shape = [m0[k] for k in ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1")]
    with M.Server(mb, mc, shape, precision=prec, max_slots=2) as srv:
        rs = srv.wait(srv.submit(p4, t, start, sc, max_evals=300, gtol=1e-6))
    with _ctx(M, mb, p4, t, mc) as c:
        rc = c.fit(start, sc, precision=prec, max_evals=300, gtol=1e-6, errors=True)
    assert rs["status"] == "converged" and rc["status"] == "converged" and rc["errors_ok"], (rs, rc)
    assert np.max(np.abs(rs["theta"][free] - rc["theta"][free]) / rc["err"][free]) < 1e-2
    assert np.array_equal(rs["theta"][~free], start[~free])
    if prec == "fp64":
        ref, gref = orc.nll_grad(mb, rs["theta"], p4, t, mc)
        _, _, _, S = orc.nll(mb, rs["theta"], p4, t, mc, diag=True)
        assert abs(rs["nll"] - ref) <= 1e-12 * max(abs(ref), 1e-3 * S)
        # near a minimum each free entry is a difference of sums of order
        # n_data that cancel (see the server tests)
        assert np.max(np.abs(rs["grad"][free] - gref[free])) <= 1e-11 * len(t)


def test_fit_recovers_the_background_fraction(M, case):
    m0, mb, th0, p4, t, mc = case
    sc = np.zeros(I.n_theta(mb))
    sc[I.theta_index(mb, "x")] = sc[I.theta_index(mb, "y")] = 1e-3
    sc[-1] = 0.05
    start = np.concatenate([th0, [0.1]])
    with _ctx(M, mb, p4, t, mc) as c:
        r = c.fit(start, sc, precision="fp64", gtol=1e-6, errors=True)
    assert r["status"] == "converged" and r["errors_ok"], r
    f_hat, sf = r["theta"][-1], r["err"][-1]
    assert 0.003 < sf < 0.05
    assert abs(f_hat - 750 / 3001) < 4 * sf, (f_hat, sf)


def test_empty_data_sample(M, case):
    m0, mb, th0, p4, t, mc = case
    with M.Context(mb, device=0) as c:
        c.load_events(M.MXA_MC, mc)
        c.set_params(np.concatenate([th0, [0.2]]))
        v, g = c.nll_grad("fp64")
    assert v == 0.0 and np.all(g == 0.0)
