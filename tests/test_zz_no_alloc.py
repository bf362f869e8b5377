"""The evaluation for callers that cannot allocate (mxa_nll_grad_noalloc),
through the C-ABI, against mxa_nll_grad on the same context and the FP64
oracle.

Both entry points launch the same kernels in the same order; only the
device memory that holds the workgroup partial sums and the slot totals
differs (the device's fixed scratch array against the context's buffers), so
the results must agree bit for bit. Two calls in a row with the second on
smaller samples show that nothing a call reads is left over from the one
before (the array keeps the last call's contents). FP64 also against the
oracle: NLL 1e-12 relative, gradient 1e-9 of max|g|.
"""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    from paper_1702_06735_amd import mixamp
    mixamp.load_library()
    return mixamp


def _sample(orc, model, theta, n_data, n_mc, seed):
    mc = I.phase_space(n_mc, seed)
    fn = lambda p, t: orc.event_terms(model, theta, p, t)
    d = I.draw_data(fn, n_data, seed + 1, model, theta, n_env=100_000, batch=1 << 16)
    return d.p4, d.t, mc


@pytest.mark.parametrize("wl", ["full", "small"])
def test_noalloc_equals_nll_grad_on_two_calls(orc, M, wl):
    W = I.WORKLOADS[wl]
    model = W.model
    theta = I.make_theta(model, I.draw_coefficients(model, W.seed_coeff))
    # a large evaluation, then a smaller one (fewer workgroups, fewer rows)
    sizes = ((4_001, 300_007, 7001), (503, 9_001, 7003))
    with M.Context(model, device=0) as ctx:
        for n_data, n_mc, seed in sizes:
            pd, td, mc = _sample(orc, model, theta, n_data, n_mc, seed)
            ctx.load_events(M.MXA_MC, mc)
            ctx.load_events(M.MXA_DATA, pd, td)
            ctx.set_params(theta)
            ref, gref = orc.nll_grad(model, theta, pd, td, mc)
            _, _, _, S = orc.nll(model, theta, pd, td, mc, diag=True)
            for prec in ("fp64", "fp32amp"):
                v0, g0, d0 = ctx.nll_grad_noalloc(prec, diag=True)
                v1, g1, d1 = ctx.nll_grad(prec, diag=True)
                v2, g2, d2 = ctx.nll_grad_noalloc(prec, diag=True)
                print(f"{wl} {n_data}/{n_mc} {prec}: noalloc {v0!r} context buffers {v1!r} "
                      f"oracle {ref!r}")
                assert v0 == v1 == v2
                assert np.array_equal(g0, g1) and np.array_equal(g0, g2)
                assert np.array_equal(d0, d1) and np.array_equal(d0, d2)
                if prec == "fp64":
                    assert abs(v0 - ref) / max(abs(ref), 1e-3 * S) <= 1e-12
                    assert np.max(np.abs(g0 - gref)) <= 1e-9 * np.max(np.abs(gref))
                else:
                    assert abs(v0 - ref) <= 1e-6 * S
                    assert np.max(np.abs(g0 - gref)) <= 1e-3 * np.max(np.abs(gref))


def test_noalloc_refuses_gram_mode(orc, M):
    model = I.MODEL_SMALL
    theta = I.make_theta(model, I.draw_coefficients(model, 101))
    pd, td, mc = _sample(orc, model, theta, 101, 2_003, 7011)
    with M.Context(model, device=0) as ctx:
        ctx.load_events(M.MXA_MC, mc)
        ctx.load_events(M.MXA_DATA, pd, td)
        ctx.set_params(theta)
        ctx.set_mc_mode(M.MXA_MC_GRAM)
        with pytest.raises(M.MixampError) as e:
            ctx.nll_grad_noalloc("fp64")
        assert e.value.code == M.MXA_EINVAL
        ctx.set_mc_mode(M.MXA_MC_DIRECT)
        v0, g0 = ctx.nll_grad_noalloc("fp64")
        v1, g1 = ctx.nll_grad("fp64")
        assert v0 == v1 and np.array_equal(g0, g1)
