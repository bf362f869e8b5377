"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark uses (the same library calls on the same sample sizes):

* the four-chain evaluation, 10,000 data / 100,000 MC;
* the headline evaluation, fourteen chains, 50,000 data / 4,000,000 MC:
  NLL and 36-component gradient against the oracle; the same sample fitted
  on the streamed fit server (masses and widths floating), whose MC walk
  runs in the benchmark's configuration;
* the differentiation form, 1,000,000 data / 4,000,000 MC: gradient against
  the oracle's dual numbers and central differences of the FP64 path;
* the precision form, 10,000,000 data / 50,000,000 MC: x, y fitted in FP64
  and with FP32 amplitudes (the same point within 1% of the errors), the FP64
  NLL against the oracle at the FP64-fitted point, the FP32-amplitude error
  against FP64, per-event terms of sampled events against the oracle.

Inputs come from the oracle's seeded generator (Philox4x32-10, GENBOD,
accept-reject by Eq. (1)). The precision form's data are 500,000 drawn
events repeated 20 times (the NLL is a plain sum over events, so the parity
check does not need them distinct; drawing 10M would take minutes of CPU)."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

MASSES = (I.MODEL_FULL["m_K"], I.MODEL_FULL["m_pi"], I.MODEL_FULL["m_pi"], I.MODEL_FULL["m_pi"])
WMAX = I.genbod_wmax(I.MODEL_FULL["m_D"], MASSES)


@pytest.fixture(scope="module")
def M():
    from paper_1702_06735_amd import mixamp
    mixamp.load_library()
    return mixamp


def _mc(orc, model, n, seed):
    """n uniform phase-space events from the oracle's generator."""
    out, first = [], 0
    while sum(len(o) for o in out) < n:
        need = n - sum(len(o) for o in out)
        _, p4, _, st = orc.generate(model, None, "mc", seed, int(need / 0.55) + 4096, WMAX,
                                    first=first, max_out=need)
        out.append(p4)
        first += int(need / 0.55) + 4096
    return np.concatenate(out).reshape(-1, 16)


def _data(orc, model, th, n, seed):
    u = _mc(orc, model, 200_000, seed + 7919)
    e = orc.event_terms(model, th, u)
    env = 1.2 * float((e[:, 0] + e[:, 1]).max())
    p4s, ts, first = [], [], 0
    while sum(len(t) for t in ts) < n:
        need = n - sum(len(t) for t in ts)
        nc = int(need / 0.004) + 65536
        _, p4, t, st = orc.generate(model, th, "data", seed, nc, WMAX, env, first=first,
                                    max_out=need)
        assert st[2] == 0, "envelope exceeded"
        p4s.append(p4.reshape(-1, 16))
        ts.append(t)
        first += nc
    return np.concatenate(p4s), np.concatenate(ts)


_WORKLOADS = {}


def _workload(orc, name, n_data=None, repeat=1):
    key = (name, n_data, repeat)
    if key not in _WORKLOADS:
        _WORKLOADS.clear()  # one workload held at a time
        _WORKLOADS[key] = _make_workload(orc, name, n_data, repeat)
    return _WORKLOADS[key]


def _make_workload(orc, name, n_data, repeat):
    W = I.WORKLOADS[name]
    m = W.model
    th = I.make_theta(m, I.draw_coefficients(m, W.seed_coeff))
    mc = _mc(orc, m, W.n_mc, W.seed_mc)
    pd, td = _data(orc, m, th, n_data or W.n_data, W.seed_data)
    if repeat > 1:
        pd, td = np.tile(pd, (repeat, 1)), np.tile(td, repeat)
    return m, th, pd, td, mc


def _load(M, m, th, pd, td, mc):
    ctx = M.Context(m, device=0)
    ctx.load_events(M.MXA_MC, mc)
    ctx.load_events(M.MXA_DATA, pd, td)
    ctx.set_params(th)
    return ctx


def _rel(v, ref, S):
    return abs(v - ref) / max(abs(ref), 1e-3 * S)


@pytest.mark.parametrize("name", ["small", "full"])
def test_evaluation_matches_oracle(orc, M, name):
    m, th, pd, td, mc = _workload(orc, name)
    ref, _, _, S = orc.nll(m, th, pd, td, mc, diag=True)
    ref_g = orc.nll_grad(m, th, pd, td, mc)[1]
    with _load(M, m, th, pd, td, mc) as ctx:
        v64, g64 = ctx.nll_grad("fp64")
        v32, g32 = ctx.nll_grad("fp32amp")
        n64 = ctx.nll("fp64")
    assert _rel(v64, ref, S) <= 1e-12 and _rel(n64, ref, S) <= 1e-12
    assert np.abs(g64 - ref_g).max() <= 1e-9 * np.abs(ref_g).max()
    assert abs(v32 - ref) <= 1e-6 * S
    assert np.abs(g32 - ref_g).max() <= 1e-3 * np.abs(ref_g).max()


def test_streamed_server_at_full_size(orc, M):
    """The streamed fit server's MC walk in the benchmark's launch
    configuration (4,000,000 MC events in 1,024 ranges, the resident grid),
    fits of the headline data sample with the masses and widths floating: at
    two points, each fit's NLL and 36-entry gradient against the oracle's (one
    evaluation per fit: a gradient tolerance no gradient reaches stops each
    fit at its start point)."""
    m, th, pd, td, mc = _workload(orc, "full")
    th2 = th.copy()
    for name, d in (("m_ks", 0.003), ("g_rho", -0.005), ("m_a1", 0.01), ("x", 0.004), ("y", -0.002)):
        th2[I.theta_index(m, name)] += d
    sc = np.full(I.n_theta(m), 1e-3)
    points = (th, th2)
    refs = [orc.nll_grad(m, t, pd, td, mc) for t in points]
    scales = [orc.nll(m, t, pd, td, mc, diag=True)[3] for t in points]
    for prec in ("fp64", "fp32amp"):
        with M.Server(m, mc, None, precision=prec, max_slots=2) as srv:
            tks = [srv.submit(pd, td, t, sc, max_evals=1, gtol=1e300) for t in points]
            out = [srv.wait(tk) for tk in tks]
        for r, t, (ref, g_ref), S in zip(out, points, refs, scales):
            assert r["n_evals"] == 1 and np.array_equal(r["theta"], t)
            gmax = np.abs(g_ref).max()
            if prec == "fp64":
                assert _rel(r["nll"], ref, S) <= 1e-12
                assert np.abs(r["grad"] - g_ref).max() <= 1e-9 * gmax
            else:
                assert abs(r["nll"] - ref) <= 1e-6 * S
                assert np.abs(r["grad"] - g_ref).max() <= 1e-3 * gmax


def test_gradient_form(orc, M):
    m, th, pd, td, mc = _workload(orc, "gradient")
    ref, ref_g = orc.nll_grad(m, th, pd, td, mc)
    with _load(M, m, th, pd, td, mc) as ctx:
        v, g = ctx.nll_grad("fp64")
        v32, g32 = ctx.nll_grad("fp32amp")
        # central differences of the FP64 path on x, y and the six masses and widths
        fd = {}
        for name in ("x", "y", "m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1"):
            j = I.theta_index(m, name)
            h = max(1e-8, 1e-6 * abs(th[j]))
            tp, tm = th.copy(), th.copy()
            tp[j] += h
            tm[j] -= h
            ctx.set_params(tp)
            fp = ctx.nll("fp64")
            ctx.set_params(tm)
            fm = ctx.nll("fp64")
            fd[j] = (fp - fm) / (2 * h)
    assert abs(v - ref) <= 1e-12 * abs(ref)
    gmax = np.abs(ref_g).max()
    assert np.abs(g - ref_g).max() <= 1e-9 * gmax
    assert np.abs(g32 - ref_g).max() <= 1e-3 * gmax
    for j, d in fd.items():
        assert abs(d - g[j]) <= 1e-5 * gmax + 1e-6 * abs(g[j]), j


def test_precision_form(orc, M):
    """FP64 NLL against the oracle at the point an FP64 fit of x, y reaches;
    x and y fitted with FP32 amplitudes within 1% of the FP64 fit's errors;
    the FP32-amplitude NLL within 1e-6 S; per-event terms of sampled events."""
    m, th, pd, td, mc = _workload(orc, "precision", n_data=500_000, repeat=20)
    assert len(td) == 10_000_000 and len(mc) == 50_000_000
    ix, iy = I.theta_index(m, "x"), I.theta_index(m, "y")
    sc = np.zeros(I.n_theta(m))
    sc[ix] = sc[iy] = 1e-3
    with _load(M, m, th, pd, td, mc) as ctx:
        rng = np.random.default_rng(3)
        for kind, p4, t in ((M.MXA_DATA, pd, td), (M.MXA_MC, mc, None)):
            terms = ctx.event_terms(kind, "fp64")
            pick = rng.choice(len(p4), 2000, replace=False)
            want = orc.event_terms(m, th, p4[pick], None if t is None else t[pick])
            got = terms[pick]
            scale = np.abs(want).max(axis=1, keepdims=True)
            assert np.all(np.abs(got - want) <= 1e-12 * scale)
        f32 = ctx.fit(th, sc, precision="fp32amp", max_evals=100, gtol=1e-12, edm_tol=1e-4)
        f64 = ctx.fit(th, sc, precision="fp64", max_evals=100, gtol=1e-12, edm_tol=1e-4,
                      errors=True)
        ctx.set_params(f64["theta"])
        v64 = ctx.nll("fp64")
        v32 = ctx.nll("fp32amp")
    assert f32["status"] == "converged" and f64["status"] == "converged" and f64["errors_ok"]
    for j in (ix, iy):
        assert abs(f32["theta"][j] - f64["theta"][j]) <= 1e-2 * f64["err"][j]
    ref, _, _, S = orc.nll(m, f64["theta"], pd, td, mc, diag=True)
    assert _rel(v64, ref, S) <= 1e-12
    assert abs(v32 - v64) <= 1e-6 * S
