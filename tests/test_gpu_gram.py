"""GPU: the MC Gram matrix (matrix-core kernel) and the Gram form of the
normalisation, against the oracle and against the direct MC pass."""

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
    W = I.WORKLOADS[request.param]
    m = W.model
    th = I.make_theta(m, I.draw_coefficients(m, W.seed_coeff))
    mc = I.phase_space(5_003, 71)
    fn = lambda p, t: orc.event_terms(m, th, p, t)
    d = I.draw_data(fn, 1_201, 72, m, th, n_env=100_000, batch=1 << 16)
    return m, th, d.p4, d.t, mc


def test_gram_matches_oracle_basis(orc, setup, M):
    m, th, pd, td, mc = setup
    B = np.array([orc.basis(m, th, e) for e in mc])         # [n, 8] chain amplitudes
    ref = B.T @ B.conj()                                     # sum_j B_k conj(B_l)
    with M.Context(m, device=0) as ctx:
        ctx.load_events(M.MXA_MC, mc)
        ctx.set_params(th)
        G = ctx.gram("fp64")
        G32 = ctx.gram("fp32amp")
    used = sorted(set(m["comp_a"]) | set(m["comp_ab"]))
    idx = np.array(used) - 1
    scale = np.abs(ref).max()
    assert np.abs(G - ref)[np.ix_(idx, idx)].max() <= 1e-12 * scale
    # chains in neither amplitude have zero rows and columns
    other = np.setdiff1d(np.arange(8), idx)
    assert np.all(G[other, :] == 0) and np.all(G[:, other] == 0)
    assert np.allclose(G, G.conj().T, rtol=0, atol=1e-13 * scale)
    assert np.abs(G32 - ref)[np.ix_(idx, idx)].max() <= 1e-5 * scale


def test_gram_mode_equals_direct_mc_pass(orc, setup, M):
    m, th, pd, td, mc = setup
    with M.Context(m, device=0) as ctx:
        ctx.load_events(M.MXA_MC, mc)
        ctx.load_events(M.MXA_DATA, pd, td)
        ctx.set_params(th)
        v_dir, g_dir, d_dir = ctx.nll_grad("fp64", diag=True)
        ctx.set_mc_mode(M.MXA_MC_GRAM)
        v_gr, g_gr, d_gr = ctx.nll_grad("fp64", diag=True)
        v_gr_nll = ctx.nll("fp64")
        v32, g32 = ctx.nll_grad("fp32amp")
        # a new point with the same lineshapes reuses the Gram
        th2 = th.copy()
        th2[0] += 0.1
        th2[I.theta_index(m, "y")] += 0.003
        ctx.set_params(th2)
        v2 = ctx.nll("fp64")
        ctx.set_mc_mode(M.MXA_MC_DIRECT)
        v2_dir = ctx.nll("fp64")
    S = d_dir[2]
    assert abs(v_gr - v_dir) <= 1e-12 * max(abs(v_dir), 1e-3 * S)
    # the FP64 NLL-only pass forms the running widths from s, the adjoint pass
    # reads them from the cache: the two agree to rounding
    assert abs(v_gr_nll - v_gr) <= 1e-13 * max(abs(v_gr), 1e-3 * S)
    assert abs(v2 - v2_dir) <= 1e-12 * max(abs(v2_dir), 1e-3 * S)
    assert d_gr[0] == pytest.approx(d_dir[0], rel=1e-12)
    n_free = 2 * (len(m["comp_a"]) + len(m["comp_ab"])) + 2
    gmax = np.abs(g_dir[:n_free]).max()
    assert np.abs(g_gr[:n_free] - g_dir[:n_free]).max() <= 1e-9 * gmax
    assert np.all(np.isnan(g_gr[n_free:]))        # masses and widths: no Gram form
    assert abs(v32 - v_dir) <= 1e-6 * S
    assert np.abs(g32[:n_free] - g_dir[:n_free]).max() <= 1e-3 * gmax
    ref = orc.nll(m, th, pd, td, mc)
    assert abs(v_gr - ref) <= 1e-12 * max(abs(ref), 1e-3 * S)
