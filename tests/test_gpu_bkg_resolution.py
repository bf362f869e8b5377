"""GPU: a background component together with a Gaussian decay-time
resolution (each data event's density at the measured time is
(1 - f) R(t) / Nhat + f Gamma_b E(Gamma_b; t)), through the C-ABI: NLL and
gradient against the oracle in both precisions, f = 0 against the resolution
model, and a fit on the fit server against the same fit on a context."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

pytestmark = pytest.mark.gpu
SIG = 0.06


@pytest.fixture(scope="module")
def M():
    from paper_1702_06735_amd import mixamp
    mixamp.load_library()
    return mixamp


@pytest.fixture(scope="module", params=["small", "full"])
def case(request, orc):
    m0 = I.MODEL_SMALL if request.param == "small" else I.MODEL_FULL
    seed = 401 if request.param == "small" else 411
    th0 = I.make_theta(m0, I.draw_coefficients(m0, seed), x=0.2, y=0.1)
    mc = I.phase_space(20_011, seed + 1)
    fn = lambda p, t: orc.event_terms(m0, th0, p, t)
    sig = I.draw_data(fn, 2_251, seed + 2, m0, th0, n_env=60_000, batch=1 << 15)
    bp, bt = I.background_events(750, seed + 3, 1.0 / 0.8)
    order = np.random.default_rng(seed + 4).permutation(3_001)
    p4 = np.concatenate([sig.p4.reshape(-1, 16), bp.reshape(-1, 16)])[order]
    t = np.concatenate([sig.t, bt])[order]
    t = t + SIG * np.random.default_rng(seed + 5).standard_normal(len(t))
    mbr = I.with_resolution(I.with_background(m0), SIG)
    return m0, mbr, th0, p4, t, mc


def _ctx(M, model, p4, t, mc):
    c = M.Context(model, device=0)
    c.load_events(M.MXA_MC, mc)
    c.load_events(M.MXA_DATA, p4, t)
    return c


def test_nll_and_gradient_match_the_oracle(orc, M, case):
    m0, mbr, th0, p4, t, mc = case
    assert (t < 0).any()
    th = np.concatenate([th0, [0.23]])
    ref, _, _, S = orc.nll(mbr, th, p4, t, mc, diag=True)
    ref_g = orc.nll_grad(mbr, th, p4, t, mc)[1]
    with _ctx(M, mbr, p4, t, mc) as c:
        c.set_params(th)
        v64, g64 = c.nll_grad("fp64")
        n64 = c.nll("fp64")
        v32, g32 = c.nll_grad("fp32amp")
        n32 = c.nll("fp32amp")
    assert abs(v64 - ref) <= 1e-12 * abs(ref) and abs(n64 - ref) <= 1e-12 * abs(ref)
    assert np.abs(g64 - ref_g).max() <= 1e-9 * np.abs(ref_g).max()
    assert abs(v32 - ref) <= 1e-6 * S and abs(n32 - ref) <= 1e-6 * S
    assert np.abs(g32 - ref_g).max() <= 1e-3 * np.abs(ref_g).max()


def test_zero_fraction_equals_the_resolution_model(M, case):
    m0, mbr, th0, p4, t, mc = case
    with _ctx(M, I.with_resolution(m0, SIG), p4, t, mc) as c:
        c.set_params(th0)
        v0, g0 = c.nll_grad("fp64")
    with _ctx(M, mbr, p4, t, mc) as c:
        c.set_params(np.concatenate([th0, [0.0]]))
        v1, g1 = c.nll_grad("fp64")
    assert abs(v1 - v0) <= 1e-12 * abs(v0)
    assert np.abs(g1[:-1] - g0).max() <= 1e-9 * np.abs(g0).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32amp"])
def test_server_fit_equals_the_context_fit(orc, M, case, prec):
    """x, y and the fraction fitted on the fit server (Nhat per tick from the
    Gram matrix) and by mxa_fit on a context: the same point to 1% of the
    errors; in FP64 the server's NLL and gradient there are the oracle's."""
    m0, mbr, th0, p4, t, mc = case
    sc = np.zeros(I.n_theta(mbr))
    sc[I.theta_index(mbr, "x")] = sc[I.theta_index(mbr, "y")] = 0.01
    sc[-1] = 0.05
    free = sc > 0
    start = np.concatenate([th0, [0.1]])
    shape = [m0[k] for k in ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1")]
    with M.Server(mbr, mc, shape, precision=prec, max_slots=2) as srv:
        rs = srv.wait(srv.submit(p4, t, start, sc, max_evals=300, gtol=1e-6))
    with _ctx(M, mbr, p4, t, mc) as c:
        rc = c.fit(start, sc, precision=prec, max_evals=300, gtol=1e-6, errors=True)
    assert rs["status"] == "converged" and rc["status"] == "converged" and rc["errors_ok"], (rs, rc)
    assert np.max(np.abs(rs["theta"][free] - rc["theta"][free]) / rc["err"][free]) < 1e-2
    assert abs(rc["theta"][-1] - 750 / 3001) < 4 * rc["err"][-1]
    if prec == "fp64":
        ref, gref = orc.nll_grad(mbr, rs["theta"], p4, t, mc)
        _, _, _, S = orc.nll(mbr, rs["theta"], p4, t, mc, diag=True)
        assert abs(rs["nll"] - ref) <= 1e-12 * max(abs(ref), 1e-3 * S)
        assert np.max(np.abs(rs["grad"][free] - gref[free])) <= 1e-11 * len(t)
