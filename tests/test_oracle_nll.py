"""Pins of the oracle's NLL and its dual-number gradient.

* Bose symmetry: exchanging the two pi- changes nothing, bit for bit.
* The NLL of a normalised density is invariant under a common complex scale
  of all coefficients; its gradient obeys the two matching Euler identities.
* x = y = 0: the NLL separates into an exponential decay-time term and a
  time-integrated amplitude term.
* Brute force on a tiny sample: the normalisation rebuilt with per-event
  adaptive quadrature over t of Eq. (1), and -sum ln p_i formed directly.
* The dual-number gradient against central finite differences.
* A fit of x, y to pseudo-data generated from the model recovers them
  (statistical; checks that the normalisation matches the generating rate).
"""

import math

import numpy as np
import pytest
from scipy import integrate, optimize

from paper_1702_06735_amd import inputs as I


def _sample(model, seed_coeff, n_data, n_mc, seed, orc, **over):
    th = I.make_theta(model, I.draw_coefficients(model, seed_coeff), **over)
    mc = I.phase_space(n_mc, seed)
    fn = lambda p, t: orc.event_terms(model, th, p, t)
    d = I.draw_data(fn, n_data, seed + 1, model, th, n_env=100_000, batch=1 << 16)
    return th, d.p4, d.t, mc


@pytest.fixture(scope="module", params=["small", "full"])
def sample(request, orc):
    W = I.WORKLOADS[request.param]
    th, pd, td, mc = _sample(W.model, W.seed_coeff, 1500, 12_000, 77, orc)
    return W.model, th, pd, td, mc


def test_bose_swap_is_bitwise(orc, sample):
    m, th, pd, td, mc = sample
    v, g = orc.nll_grad(m, th, pd, td, mc)
    vs, gs = orc.nll_grad(m, th, I.swap_pions(pd), td, I.swap_pions(mc))
    assert v == vs
    assert np.array_equal(g, gs)
    assert orc.nll(m, th, pd, td, mc) == orc.nll(m, th, I.swap_pions(pd), td, I.swap_pions(mc))


def test_thread_count_does_not_change_result(orc, sample):
    m, th, pd, td, mc = sample
    assert orc.nll(m, th, pd, td, mc, nthreads=1) == orc.nll(m, th, pd, td, mc, nthreads=4)


def _coeff_slots(m):
    return 2 * (len(m["comp_a"]) + len(m["comp_ab"]))


def test_common_coefficient_scale_and_phase(orc, sample):
    m, th, pd, td, mc = sample
    nc = _coeff_slots(m)
    v0, _, _, S = orc.nll(m, th, pd, td, mc, diag=True)
    c = th[0:nc:2] + 1j * th[1:nc:2]
    for lam in [2.5, 0.3 * np.exp(1j * 1.1), np.exp(-2j)]:
        th2 = th.copy()
        cl = c * lam
        th2[0:nc:2], th2[1:nc:2] = cl.real, cl.imag
        assert abs(orc.nll(m, th2, pd, td, mc) - v0) <= 1e-12 * S


def test_euler_identities_of_gradient(orc, sample):
    m, th, pd, td, mc = sample
    nc = _coeff_slots(m)
    _, g = orc.nll_grad(m, th, pd, td, mc)
    u, v = th[0:nc:2], th[1:nc:2]
    gu, gv = g[0:nc:2], g[1:nc:2]
    norm = np.abs(g[:nc]).max() * np.abs(th[:nc]).max() * nc
    assert abs(np.sum(u * gu + v * gv)) <= 1e-11 * norm       # scale
    assert abs(np.sum(-v * gu + u * gv)) <= 1e-11 * norm      # phase


def test_no_mixing_separates(orc, sample):
    m, th, pd, td, mc = sample
    th0 = th.copy()
    th0[I.theta_index(m, "x")] = 0.0
    th0[I.theta_index(m, "y")] = 0.0
    G = 1.0 / m["tau"]
    a2d = orc.event_terms(m, th0, pd, td)[:, 0]
    a2m = orc.event_terms(m, th0, mc)[:, 0]
    n = len(td)
    time_part = np.sum(G * td - math.log(G))
    amp_part = n * math.log(np.mean(a2m)) - np.sum(np.log(a2d))
    v, _, _, S = orc.nll(m, th0, pd, td, mc, diag=True)
    assert abs(v - (time_part + amp_part)) <= 1e-12 * S


def _amplitudes(orc, m, th, ev):
    nA = len(m["comp_a"])
    nc = _coeff_slots(m)
    c = th[0:nc:2] + 1j * th[1:nc:2]
    B = orc.basis(m, th, ev)
    A = sum(c[j] * B[k - 1] for j, k in enumerate(m["comp_a"]))
    Ab = sum(c[nA + j] * B[k - 1] for j, k in enumerate(m["comp_ab"]))
    return A, Ab


def test_brute_force_normalisation_tiny_sample(orc):
    m = I.MODEL_FULL
    th = I.make_theta(m, I.draw_coefficients(m, 9), x=0.03, y=-0.04)
    G = 1.0 / m["tau"]
    x, y = th[I.theta_index(m, "x")], th[I.theta_index(m, "y")]
    ev = I.phase_space(9, 123)
    pd, mc = ev[:4], ev[4:]
    td = np.array([0.1, 0.7, 1.9, 0.02])
    tmax = 80.0 / (G * (1.0 - abs(y)))
    norms = []
    for e in mc:
        A, Ab = _amplitudes(orc, m, th, e)
        f = lambda t: math.exp(-G * t) * orc.rate(A, Ab, x, y, G, t)
        norms.append(integrate.quad(f, 0.0, tmax, epsabs=0, epsrel=1e-13, limit=400)[0])
    nhat = math.fsum(norms) / len(norms)
    terms = []
    for e, t in zip(pd, td):
        A, Ab = _amplitudes(orc, m, th, e)
        p = math.exp(-G * t) * orc.rate(A, Ab, x, y, G, t) / nhat
        terms.append(-math.log(p))
    v, nh, _, S = orc.nll(m, th, pd, td, mc, diag=True)
    assert nh == pytest.approx(nhat, rel=1e-11)
    assert abs(v - math.fsum(terms)) <= 1e-11 * S


def test_gradient_matches_central_differences(orc, sample):
    m, th, pd, td, mc = sample
    _, g = orc.nll_grad(m, th, pd, td, mc)
    fd = np.empty_like(g)
    for i in range(th.size):
        h = 1e-6 * max(abs(th[i]), 1e-2)
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (orc.nll(m, tp, pd, td, mc) - orc.nll(m, tm, pd, td, mc)) / (2 * h)
    assert np.all(np.abs(fd - g) <= 2e-5 * np.abs(g).max())


def test_domain_errors(orc, sample):
    m, th, pd, td, mc = sample
    bad = th.copy()
    bad[I.theta_index(m, "y")] = 1.0
    with pytest.raises(orc.OracleError):
        orc.nll(m, bad, pd, td, mc)
    bad = th.copy()
    bad[I.theta_index(m, "m_rho")] = 0.2
    with pytest.raises(orc.OracleError):
        orc.nll(m, bad, pd, td, mc)
    bad = th.copy()
    bad[I.theta_index(m, "g_a1")] = -0.1
    with pytest.raises(orc.OracleError):
        orc.nll(m, bad, pd, td, mc)


@pytest.mark.slow
def test_fit_recovers_mixing_parameters(orc):
    """Pseudo-data generated with the oracle's Eq. (1); the fit uses the
    oracle's normalisation. A normalisation that is not the integral of the
    generating rate (a wrong time integral, a missing n ln Nhat) biases x, y
    by many standard deviations."""
    m = I.MODEL_SMALL
    x0, y0 = 0.05, 0.08   # large mixing so that the test has power at 20k events
    th, pd, td, mc = _sample(m, 101, 20_000, 300_000, 991, orc, x=x0, y=y0)
    ix, iy = I.theta_index(m, "x"), I.theta_index(m, "y")

    def f(p):
        t = th.copy()
        t[ix], t[iy] = p
        v, g = orc.nll_grad(m, t, pd, td, mc)
        return v, np.array([g[ix], g[iy]])

    res = optimize.minimize(f, [0.0, 0.0], jac=True, method="L-BFGS-B",
                            bounds=[(-0.5, 0.5), (-0.5, 0.5)],
                            options=dict(gtol=1e-8, ftol=1e-15))
    xh, yh = res.x
    # covariance from the numerical Hessian of the gradient
    h = 1e-4
    H = np.empty((2, 2))
    for i in range(2):
        e = np.zeros(2)
        e[i] = h
        H[:, i] = (f(res.x + e)[1] - f(res.x - e)[1]) / (2 * h)
    cov = np.linalg.inv(0.5 * (H + H.T))
    sx, sy = math.sqrt(cov[0, 0]), math.sqrt(cov[1, 1])
    assert abs(xh - x0) < 5 * sx, (xh, sx)
    assert abs(yh - y0) < 5 * sy, (yh, sy)
    # the test has power: the truth is far from zero in units of sigma
    assert abs(x0) > 5 * sx or abs(y0) > 5 * sy
