"""GPU: the streamed fit server, whose fits float the masses and widths and
whose every tick reads the shared MC sample once for all active fits (the
Sec. 3.1 normalisation with the lineshapes recomputed per fit), through the
C-ABI; and the gradient the fit results report."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

pytestmark = pytest.mark.gpu

MODEL = I.MODEL_FULL
SHAPE = [MODEL[k] for k in ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1")]
SHAPE_NAMES = ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1")


@pytest.fixture(scope="module")
def M():
    from paper_1702_06735_amd import mixamp
    mixamp.load_library()
    return mixamp


def scales(model, shapes=True):
    """Coefficients 0.05 except the a1 S-wave one of Abar_f (held fixed: global
    phase and scale), x, y 1e-3, masses and widths 2e-3 GeV when floating."""
    sc = np.zeros(I.n_theta(model))
    nc = len(model["comp_a"]) + len(model["comp_ab"])
    sc[:2 * nc] = 0.05
    j = len(model["comp_a"]) + model["comp_ab"].index(5)
    sc[2 * j:2 * j + 2] = 0.0
    sc[I.theta_index(model, "x")] = sc[I.theta_index(model, "y")] = 1e-3
    if shapes:
        for k in SHAPE_NAMES:
            sc[I.theta_index(model, k)] = 2e-3
    return sc


@pytest.fixture(scope="module")
def toy(orc):
    th = I.make_theta(MODEL, I.draw_coefficients(MODEL, 211))
    mc = I.phase_space(60_000, 612)
    fn = lambda p, t: orc.event_terms(MODEL, th, p, t)
    samples = []
    for i, n in enumerate([5_000, 2_000, 7_500, 3_000]):
        d = I.draw_data(fn, n, 720 + i, MODEL, th, n_env=100_000, batch=1 << 16)
        samples.append((d.p4, d.t))
    rng = np.random.default_rng(5)
    start = th.copy()
    start[:2 * 14] += rng.normal(0, 0.02, 28) * (scales(MODEL)[:28] > 0)
    start[I.theta_index(MODEL, "x")] = 0.0
    start[I.theta_index(MODEL, "y")] = 0.0
    for k, d in zip(SHAPE_NAMES, (0.004, -0.003, 0.005, 0.006, -0.01, 0.02)):
        start[I.theta_index(MODEL, k)] += d
    return th, start, mc, samples


def _check_against_oracle(orc, r, p4, t, mc, grad=True):
    ref, g_ref = orc.nll_grad(MODEL, r["theta"], p4, t, mc)
    _, _, _, S = orc.nll(MODEL, r["theta"], p4, t, mc, diag=True)
    assert abs(r["nll"] - ref) <= 1e-12 * max(abs(ref), 1e-3 * S), (r["nll"], ref)
    if grad:
        g = r["grad"]
        scale = np.max(np.abs(g_ref))
        assert np.all(np.abs(g - g_ref) <= 1e-9 * scale), np.max(np.abs(g - g_ref)) / scale


def test_streamed_fits_match_the_oracle_fp64(orc, toy, M):
    """Several fits share each tick's MC pass; at every fit's reported point
    the NLL and the full 36-entry gradient (masses and widths included) agree
    with the oracle's."""
    th, start, mc, samples = toy
    with M.Server(MODEL, mc, None, precision="fp64", max_slots=4) as srv:
        tickets = [srv.submit(p4, t, start, scales(MODEL), max_evals=8, gtol=1e-12)
                   for p4, t in samples[:3]]
        out = [srv.wait(tk) for tk in tickets]
    for r, (p4, t) in zip(out, samples[:3]):
        assert r["status"] in ("converged", "max_evals"), r["status"]
        # the masses and widths moved: they float
        k = [I.theta_index(MODEL, s) for s in SHAPE_NAMES]
        assert np.any(r["theta"][k] != start[k])
        _check_against_oracle(orc, r, p4, t, mc)


def test_streamed_fit_with_fp32_amplitudes(orc, toy, M):
    th, start, mc, samples = toy
    p4, t = samples[0]
    with M.Server(MODEL, mc, None, precision="fp32amp", max_slots=2) as srv:
        r = srv.wait(srv.submit(p4, t, start, scales(MODEL), max_evals=8, gtol=1e-12))
    ref = orc.nll(MODEL, r["theta"], p4, t, mc)
    _, _, _, S = orc.nll(MODEL, r["theta"], p4, t, mc, diag=True)
    assert abs(r["nll"] - ref) <= 1e-6 * S


def test_streamed_result_is_the_same_alone_and_in_the_mix(toy, M):
    th, start, mc, samples = toy

    def run(jobs):
        with M.Server(MODEL, mc, None, precision="fp32amp", max_slots=8) as srv:
            tks = [srv.submit(p4, t, start, scales(MODEL), max_evals=30) for p4, t in jobs]
            return [srv.wait(tk) for tk in tks]

    alone = run(samples[:1])
    mixed = run(samples)
    assert np.array_equal(alone[0]["theta"], mixed[0]["theta"])
    assert alone[0]["nll"] == mixed[0]["nll"]
    assert alone[0]["n_evals"] == mixed[0]["n_evals"]
    assert np.array_equal(alone[0]["grad"], mixed[0]["grad"])


def test_floating_shapes_fit_converges(orc, toy, M):
    th, start, mc, samples = toy
    p4, t = samples[2]
    with M.Server(MODEL, mc, None, precision="fp64", max_slots=2) as srv:
        r = srv.wait(srv.submit(p4, t, start, scales(MODEL), max_evals=600, gtol=1e-3,
                                edm_tol=1e-5))
    assert r["status"] == "converged", r
    _, _, _, S = orc.nll(MODEL, r["theta"], p4, t, mc, diag=True)
    # at least as good as the generating point
    assert r["nll"] <= orc.nll(MODEL, th, p4, t, mc) + 1e-6 * S
    fixed = scales(MODEL) == 0
    assert np.array_equal(r["theta"][fixed], start[fixed])
    _check_against_oracle(orc, r, p4, t, mc, grad=False)


def test_streamed_with_fixed_shapes_agrees_with_the_gram_server(orc, toy, M):
    """With the masses and widths fixed, the streamed server's MC sums and the
    Gram form of the fixed-lineshape server give the same NLL at the same
    point (one evaluation: a gradient tolerance no gradient can exceed stops
    each fit at theta0)."""
    th, start, mc, samples = toy
    p4, t = samples[1]
    st = start.copy()
    for k, v in zip(SHAPE_NAMES, SHAPE):
        st[I.theta_index(MODEL, k)] = v
    sc = scales(MODEL, shapes=False)
    out = []
    for shape in (None, SHAPE):
        with M.Server(MODEL, mc, shape, precision="fp64", max_slots=2) as srv:
            out.append(srv.wait(srv.submit(p4, t, st, sc, max_evals=1, gtol=1e300)))
    a, b = out
    assert a["n_evals"] == b["n_evals"] == 1
    assert np.array_equal(a["theta"], st) and np.array_equal(b["theta"], st)
    _, _, _, S = orc.nll(MODEL, a["theta"], p4, t, mc, diag=True)
    assert abs(a["nll"] - b["nll"]) <= 1e-12 * max(abs(a["nll"]), 1e-3 * S)
    n_c = 2 * 14 + 2  # coefficients, x and y: gradient entries both servers give
    ga, gb = a["grad"][:n_c], b["grad"][:n_c]
    assert np.all(np.abs(ga - gb) <= 1e-9 * np.max(np.abs(ga)))
    # the fixed-lineshape server has no lineshape gradient
    assert np.all(np.isnan(b["grad"][n_c:]))
    assert np.all(np.isfinite(a["grad"]))


def test_gram_server_gradient_matches_the_oracle(orc, toy, M):
    th, start, mc, samples = toy
    p4, t = samples[0]
    st = start.copy()
    for k, v in zip(SHAPE_NAMES, SHAPE):
        st[I.theta_index(MODEL, k)] = v
    with M.Server(MODEL, mc, SHAPE, precision="fp64", max_slots=2) as srv:
        r = srv.wait(srv.submit(p4, t, st, scales(MODEL, shapes=False), max_evals=6, gtol=1e-12))
    ref, g_ref = orc.nll_grad(MODEL, r["theta"], p4, t, mc)
    n_c = 2 * 14 + 2
    scale = np.max(np.abs(g_ref[:n_c]))
    assert np.all(np.abs(r["grad"][:n_c] - g_ref[:n_c]) <= 1e-9 * scale)


def test_single_context_fit_reports_its_gradient(orc, toy, M):
    th, start, mc, samples = toy
    p4, t = samples[1]
    with M.Context(MODEL, device=0) as ctx:
        ctx.load_events(M.MXA_MC, mc)
        ctx.load_events(M.MXA_DATA, p4, t)
        r = ctx.fit(start, scales(MODEL), precision="fp64", max_evals=5, gtol=1e-12)
    _check_against_oracle(orc, r, p4, t, mc)


@pytest.mark.parametrize("n_mc", [5, 1_000, 2_500])
def test_streamed_small_model_small_mc_and_fits_finishing_apart(orc, M, n_mc):
    """The four-component model; MC samples of fewer events than the walk has
    ranges (empty ranges), or not a multiple of them; three fits that stop
    after different numbers of evaluations, so the active list has gaps
    (slots 0 and 2 go on after slot 1 has finished)."""
    model = I.MODEL_SMALL
    th = I.make_theta(model, I.draw_coefficients(model, 101))
    mc = I.phase_space(n_mc, 102)
    fn = lambda p, t: orc.event_terms(model, th, p, t)
    data = [I.draw_data(fn, n, 110 + i, model, th, n_env=20_000, batch=1 << 14)
            for i, n in enumerate([400, 250, 700])]
    sc = np.zeros(I.n_theta(model))
    nc = len(model["comp_a"]) + len(model["comp_ab"])
    sc[2:2 * nc] = 0.05  # the first coefficient fixed (global phase and scale)
    sc[I.theta_index(model, "x")] = sc[I.theta_index(model, "y")] = 1e-3
    for k in SHAPE_NAMES:
        sc[I.theta_index(model, k)] = 2e-3
    with M.Server(model, mc, None, precision="fp64", max_slots=3) as srv:
        tks = [srv.submit(d.p4, d.t, th, sc, max_evals=m, gtol=1e-12)
               for d, m in zip(data, (7, 2, 11))]
        out = [srv.wait(tk) for tk in tks]
    for r, d in zip(out, data):
        ref, g_ref = orc.nll_grad(model, r["theta"], d.p4, d.t, mc)
        _, _, _, S = orc.nll(model, r["theta"], d.p4, d.t, mc, diag=True)
        assert abs(r["nll"] - ref) <= 1e-12 * max(abs(ref), 1e-3 * S), (r["nll"], ref)
        scale = np.max(np.abs(g_ref))
        assert np.all(np.abs(r["grad"] - g_ref) <= 1e-9 * scale)
    assert [r["n_evals"] for r in out][1] < [r["n_evals"] for r in out][2]


def test_streamed_device_events_match_the_oracle(orc, toy, M):
    """The streamed server reads events handed over on the device in place
    (events_on_device): the fit is the one of the same events from host
    memory, bit for bit, and its NLL and gradient are the oracle's."""
    import torch
    th, start, mc, samples = toy
    p4, t = samples[1]
    dp = torch.from_numpy(np.ascontiguousarray(p4, dtype=np.float64)).to("cuda:0")
    dt = torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).to("cuda:0")
    with M.Server(MODEL, mc, None, precision="fp64", max_slots=2) as srv:
        a = srv.wait(srv.submit(p4, t, start, scales(MODEL), max_evals=8, gtol=1e-12), release=True)
        b = srv.wait(srv.submit(dp, dt, start, scales(MODEL), max_evals=8, gtol=1e-12), release=True)
    assert np.array_equal(a["theta"], b["theta"]) and a["nll"] == b["nll"]
    _check_against_oracle(orc, b, p4, t, mc)
