"""GPU: the fit server (continuous batching of toy fits with a shared MC Gram
matrix), through the C-ABI."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

pytestmark = pytest.mark.gpu

MODEL = I.MODEL_FULL
SHAPE = [MODEL[k] for k in ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1")]


@pytest.fixture(scope="module")
def M():
    from paper_1702_06735_amd import mixamp
    mixamp.load_library()
    return mixamp


def scales(model):
    """Step scales: coefficients 0.05 except the a1 S-wave one of Abar_f, which
    is held fixed (global phase and scale), x, y 1e-3, lineshapes fixed."""
    sc = np.zeros(I.n_theta(model))
    nc = len(model["comp_a"]) + len(model["comp_ab"])
    sc[:2 * nc] = 0.05
    j = len(model["comp_a"]) + model["comp_ab"].index(5)
    sc[2 * j:2 * j + 2] = 0.0
    sc[I.theta_index(model, "x")] = sc[I.theta_index(model, "y")] = 1e-3
    return sc


@pytest.fixture(scope="module")
def toy(orc):
    th = I.make_theta(MODEL, I.draw_coefficients(MODEL, 201))
    mc = I.phase_space(60_000, 602)
    fn = lambda p, t: orc.event_terms(MODEL, th, p, t)
    samples = []
    for i, n in enumerate([6_000, 2_500, 9_000, 4_000]):
        d = I.draw_data(fn, n, 700 + i, MODEL, th, n_env=100_000, batch=1 << 16)
        samples.append((d.p4, d.t))
    rng = np.random.default_rng(3)
    start = th.copy()
    start[:2 * 14] += rng.normal(0, 0.02, 28) * (scales(MODEL)[:28] > 0)
    start[I.theta_index(MODEL, "x")] = 0.0
    start[I.theta_index(MODEL, "y")] = 0.0
    return th, start, mc, samples


def a_scales(model):
    """A_f's coefficients and x, y free, Abar_f fixed: a well-conditioned fit
    (Abar_f enters the rate only through O(x, y) terms)."""
    sc = np.zeros(I.n_theta(model))
    sc[:2 * len(model["comp_a"])] = 0.05
    sc[I.theta_index(model, "x")] = sc[I.theta_index(model, "y")] = 1e-3
    return sc


def test_fit_converges_and_agrees_with_oracle(orc, toy, M):
    th, start, mc, samples = toy
    p4, t = samples[0]
    with M.Server(MODEL, mc, SHAPE, precision="fp64", max_slots=4) as srv:
        r = srv.wait(srv.submit(p4, t, start, a_scales(MODEL), max_evals=400, gtol=1e-4))
    assert r["status"] == "converged", r
    ref, gref = orc.nll_grad(MODEL, r["theta"], p4, t, mc)
    _, _, _, S = orc.nll(MODEL, r["theta"], p4, t, mc, diag=True)
    assert abs(r["nll"] - ref) <= 1e-12 * max(abs(ref), 1e-3 * S)
    # the reported gradient at the best point is the oracle's. At a minimum
    # each free entry is the difference of a data sum and a normalisation sum,
    # each of order n_data, that cancel: FP64 rounding of those sums (1e-12
    # relative, the Gram form against the oracle's direct sum) leaves absolute
    # errors of order 1e-12 n_data
    free = a_scales(MODEL) > 0
    assert np.max(np.abs(r["grad"][free] - gref[free])) <= 1e-11 * len(t)
    # a stationary point of the oracle's NLL in the free parameters (to what
    # the NLL's FP64 rounding lets a line search resolve)
    assert np.max(np.abs(gref[free] * a_scales(MODEL)[free])) < 1e-3
    # the minimum is at least as good as the generating point
    assert r["nll"] <= orc.nll(MODEL, th, p4, t, mc) + 1e-6 * S
    # fixed parameters did not move
    fixed = a_scales(MODEL) == 0
    assert np.array_equal(r["theta"][fixed], start[fixed])


def _run(M, mc, jobs, **kw):
    with M.Server(MODEL, mc, SHAPE, **kw) as srv:
        tickets = [srv.submit(p4, t, th0, scales(MODEL), max_evals=120) for p4, t, th0 in jobs]
        out = [srv.wait(tk) for tk in tickets]
        stats = srv.stats()
    return out, stats


def test_result_is_the_same_alone_and_in_the_mix(toy, M):
    th, start, mc, samples = toy
    jobs = [(p4, t, start) for p4, t in samples]
    alone, _ = _run(M, mc, jobs[:1], precision="fp32amp", max_slots=8)
    mixed, stats = _run(M, mc, jobs, precision="fp32amp", max_slots=8)
    assert np.array_equal(alone[0]["theta"], mixed[0]["theta"])
    assert alone[0]["nll"] == mixed[0]["nll"]
    assert alone[0]["n_evals"] == mixed[0]["n_evals"]
    assert stats["ticks"] < sum(r["n_evals"] for r in mixed)   # evaluations were batched


def _held(n):
    """Device bytes of an FP32 fit of n events while it is admitted: its basis
    and times (16 FP32 columns for the eight chains + 8 B = 72 B per event on n
    rounded up to 64) and the staging (the events and times as copied, 136 B
    per event, and the tier-0 record the basis is computed from, 25 FP32
    columns, each part rounded up to 256 B, plus 256 B)."""
    r = lambda b: (b + 255) // 256 * 256
    ld = (n + 63) // 64 * 64
    return 72 * ld + r(128 * n) + r(8 * n) + 256 + r(100 * ld)


def _footprint(n):
    return 72 * ((n + 63) // 64 * 64)


def test_admission_under_a_small_budget(toy, M):
    th, start, mc, samples = toy
    jobs = [(p4, t, start) for p4, t in samples] * 2
    sizes = [len(t) for _, t, _ in jobs]
    budget = _held(max(sizes))                # just room to admit the largest fit
    free, fstats = _run(M, mc, jobs, precision="fp32amp", max_slots=8)
    tight, stats = _run(M, mc, jobs, precision="fp32amp", max_slots=8, hbm_budget=budget)
    for a, b in zip(free, tight):
        assert np.array_equal(a["theta"], b["theta"]) and a["nll"] == b["nll"]
    assert stats["hbm_used"] == 0
    # the budget bound what was held at every moment ...
    assert 0 < stats["hbm_peak"] <= budget < fstats["hbm_peak"]
    # ... and so the concurrency: k fits are active together only if the
    # footprints of k - 1 of them and the admission of the k-th fit in the
    # budget (least for the k smallest, the smallest admitted last)
    order = sorted(sizes)
    bound = max(k for k in range(1, len(sizes) + 1)
                if sum(_footprint(n) for n in order[:k]) - _footprint(order[0]) + _held(order[0])
                <= budget)
    assert stats["active_peak"] <= bound < fstats["active_peak"]
    with M.Server(MODEL, mc, SHAPE, precision="fp32amp", hbm_budget=1 << 19) as srv:
        with pytest.raises(M.MixampError) as e:
            srv.submit(samples[0][0], samples[0][1], start, scales(MODEL))
        assert e.value.code == M.MXA_ENOMEM


def test_graph_replay_equals_direct_launches(toy, M):
    th, start, mc, samples = toy
    p4, t = samples[1]
    outs = []
    for graph in (True, False):
        with M.Server(MODEL, mc, SHAPE, precision="fp32amp", max_slots=2) as srv:
            srv.set_graph(graph)
            outs.append(srv.wait(srv.submit(p4, t, start, scales(MODEL), max_evals=60)))
    assert np.array_equal(outs[0]["theta"], outs[1]["theta"]) and outs[0]["nll"] == outs[1]["nll"]


def test_cancel_and_unknown_ticket(toy, M):
    th, start, mc, samples = toy
    p4, t = samples[2]
    with M.Server(MODEL, mc, SHAPE, precision="fp32amp", max_slots=1) as srv:
        t1 = srv.submit(p4, t, start, scales(MODEL), max_evals=100000, gtol=1e-30)
        t2 = srv.submit(p4, t, start, scales(MODEL))
        srv.cancel(t2)                          # still queued behind t1
        srv.cancel(t1)                          # running
        assert srv.wait(t1)["status"] == "cancelled"
        assert srv.wait(t2)["status"] == "cancelled"
        with pytest.raises(M.MixampError) as e:
            srv.poll(123456)
        assert e.value.code == M.MXA_ENOTFOUND


def test_edm_rule_converges_with_fp32_amplitudes(orc, toy, M):
    """The toy fits of Sec. 4 keep the amplitude model fixed and float x and
    y. With FP32 amplitudes the gradient carries rounding noise, so a tight
    gradient test cannot be met; the estimated-distance rule stops the fit,
    at the FP64 fit's minimum within 1e-3 in the NLL."""
    th, start, mc, samples = toy
    p4, t = samples[2]
    sc = np.zeros(I.n_theta(MODEL))
    sc[I.theta_index(MODEL, "x")] = sc[I.theta_index(MODEL, "y")] = 1e-3
    with M.Server(MODEL, mc, SHAPE, precision="fp32amp", max_slots=2) as srv:
        r32 = srv.wait(srv.submit(p4, t, th, sc, max_evals=100, gtol=1e-12, edm_tol=1e-4))
    with M.Server(MODEL, mc, SHAPE, precision="fp64", max_slots=2) as srv:
        r64 = srv.wait(srv.submit(p4, t, th, sc, max_evals=100, gtol=1e-7))
    assert r32["status"] == "converged" and r32["n_evals"] < 40, r32
    assert r64["status"] == "converged", r64
    n32 = orc.nll(MODEL, r32["theta"], p4, t, mc)
    n64 = orc.nll(MODEL, r64["theta"], p4, t, mc)
    assert abs(n32 - n64) < 1e-3


def test_device_events_equal_host_events(toy, M):
    """Events handed over in place on the device (events_on_device: the
    admission reads them there, no copy) give the fit of the same events
    submitted from host memory, bit for bit; host memory flagged as device
    memory is refused with MXA_EINVAL."""
    import ctypes as C

    import torch
    th, start, mc, samples = toy
    p4, t = samples[1]
    dp = torch.from_numpy(np.ascontiguousarray(p4, dtype=np.float64)).to("cuda:0")
    dt = torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).to("cuda:0")
    with M.Server(MODEL, mc, SHAPE, precision="fp64", max_slots=2) as srv:
        a = srv.wait(srv.submit(p4, t, start, scales(MODEL), max_evals=60), release=True)
        b = srv.wait(srv.submit(dp, dt, start, scales(MODEL), max_evals=60), release=True)
        assert np.array_equal(a["theta"], b["theta"]) and a["nll"] == b["nll"]
        assert a["n_evals"] == b["n_evals"]
        hp = np.ascontiguousarray(p4, dtype=np.float64).reshape(-1, 16)
        ht = np.ascontiguousarray(t, dtype=np.float64)
        sc = np.ascontiguousarray(scales(MODEL))
        st = np.ascontiguousarray(start, dtype=np.float64)
        pd = lambda x: x.ctypes.data_as(C.POINTER(C.c_double))
        req = M.FitRequest(pd(hp), pd(ht), hp.shape[0], pd(st), pd(sc), 60, 1e-3, 0.0, 0.0, 0, 0, 1)
        ticket = C.c_uint64()
        assert srv._lib.mxa_fit_submit(srv._h, C.byref(req), C.byref(ticket)) == M.MXA_EINVAL


def test_general_chain_set_agrees_with_oracle(orc, M):
    """A model whose chain set is neither of the two presets (A_f = chains 1
    and 6, Abar_f = chains 5 and 7) runs the general kernels, with a basis of
    all eight chains: a converged FP64 server fit's NLL and gradient are the
    oracle's at the fitted point."""
    model = dict(I.MODEL_FULL, name="general", comp_a=[1, 6], comp_ab=[5, 7])
    th = I.make_theta(model, I.draw_coefficients(model, 211))
    mc = I.phase_space(40_000, 612)
    fn = lambda p, t: orc.event_terms(model, th, p, t)
    d = I.draw_data(fn, 4_000, 713, model, th, n_env=60_000, batch=1 << 16)
    shape = [model[k] for k in ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1")]
    sc = a_scales(model)
    start = th.copy()
    start[I.theta_index(model, "x")] = start[I.theta_index(model, "y")] = 0.0
    with M.Server(model, mc, shape, precision="fp64", max_slots=2) as srv:
        r = srv.wait(srv.submit(d.p4, d.t, start, sc, max_evals=300, gtol=1e-4), release=True)
    assert r["status"] == "converged", r
    ref, gref = orc.nll_grad(model, r["theta"], d.p4, d.t, mc)
    _, _, _, S = orc.nll(model, r["theta"], d.p4, d.t, mc, diag=True)
    assert abs(r["nll"] - ref) <= 1e-12 * max(abs(ref), 1e-3 * S)
    free = sc > 0
    assert np.max(np.abs(r["grad"][free] - gref[free])) <= 1e-11 * len(d.t)
