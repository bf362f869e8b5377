"""Pin of the oracle's chain assembly (Sec. 3, Eq. (2) and the Fig. 2
topologies): which spin factor, D-vertex barrier and lineshapes each of the
eight decay chains multiplies, the Bose sum over the two pi-, and which chains
A_f and Abar_f take.

The oracle's ``basis`` builds the chains internally. Here every chain is
rebuilt from pieces that are pinned on their own -- the raw spin factors and
D-vertex momenta (``test_oracle_spin.py``: explicit rest-frame construction),
the barrier factors (spherical Hankel functions) and the lineshapes (pole
value, Lorentzian integral, power laws; ``test_oracle_lineshapes.py``) -- and
the invariant masses are recomputed here from the four-momenta. The chain
table below is written from the model description (the basis table of the
reading of Sec. 3), not from the oracle's source, so a wrong barrier, a wrong
sub-resonance mass in a three-body lineshape, a swapped constant or a chain in
the wrong amplitude fails one of these tests.
"""

import math

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

FULL, SMALL = I.MODEL_FULL, I.MODEL_SMALL
MD, MK, MPI, R = FULL["m_D"], FULL["m_K"], FULL["m_pi"], FULL["r"]

# Membership of the two amplitudes (chain indices 1..8), per model.
MEMBERS = {
    "fourteen-component": ([1, 2, 3, 4, 7, 8], [1, 2, 3, 4, 5, 6, 7, 8]),
    "four-component": ([1, 4], [5, 2]),
}


def mdot(a, b):
    return a[0] * b[0] - a[1:] @ b[1:]


def invariants(ev, sigma):
    """s(K+ pi_s), s(pi+ pi_o), s(K+ pi_s pi+), s(pi- pi+ pi-) from the momenta."""
    k, pa, pip, pb = (np.asarray(ev[i], dtype=float) for i in range(4))
    ps, po = (pa, pb) if sigma == 0 else (pb, pa)
    return np.array([mdot(k + ps, k + ps), mdot(pip + po, pip + po),
                     mdot(k + ps + pip, k + ps + pip), mdot(pa + pip + pb, pa + pip + pb)])


def kallen_q(M2, ma, mb):
    """Break-up momentum of a system of mass squared M2 into ma, mb."""
    v = (M2 - (ma + mb) ** 2) * (M2 - (ma - mb) ** 2) / (4.0 * M2)
    return math.sqrt(max(v, 0.0))


def chains(orc, model, th, ev, sigma):
    """b_1 .. b_8 of one Bose configuration from the separately pinned pieces.

    Chain k: spin factor x D-vertex barrier F_L(q_D) x lineshapes
      1 VV S-wave   SF_S                 LS_K* LS_rho
      2 VV P-wave   SF_P F_1(q_D,VV)     LS_K* LS_rho
      3 VV D-wave   SF_D F_2(q_D,VV)     LS_K* LS_rho
      4 SV          SF_SV F_1(q_D,VV)    LS_rho
      5 a1 S-wave   SF_a1S F_1(q_D,a1)   LS_a1(L=0) LS_rho
      6 a1 D-wave   SF_a1D F_1(q_D,a1)   LS_a1(L=2) LS_rho
      7 K1(1270)    SF_K1 F_1(q_D,K1)    LS_K1(1270) LS_K*
      8 K1(1400)    SF_K1 F_1(q_D,K1)    LS_K1(1400) LS_K*
    Two-body lineshapes at s(K+ pi_s) and s(pi+ pi_o); a1 at s(3 pi) with the
    rho0 of this configuration (s(pi+ pi_o)) and the bachelor pi_s, q0 at the
    nominal rho0 mass; K1 at s(K+ pi_s pi+) with the K*0 of this configuration
    (s(K+ pi_s)) and the pi+, q0 at the nominal K*0 mass, L = 0.
    """
    sf, qd, s = orc.spin_factors(ev, MD, MK, MPI)
    sf, qd, s = sf[sigma], qd[sigma], s[sigma]
    s_kpi, s_pipi, s_kpipi, s_3pi = s
    m_ks, g_ks = th[I.theta_index(model, "m_ks")], th[I.theta_index(model, "g_ks")]
    m_rho, g_rho = th[I.theta_index(model, "m_rho")], th[I.theta_index(model, "g_rho")]
    m_a1, g_a1 = th[I.theta_index(model, "m_a1")], th[I.theta_index(model, "g_a1")]
    ks = orc.ls_two_body(s_kpi, m_ks, g_ks, MK, MPI, R)
    rho = orc.ls_two_body(s_pipi, m_rho, g_rho, MPI, MPI, R)
    a1s = orc.ls_three_body(0, s_3pi, s_pipi, MPI, m_a1, g_a1, model["m_rho_ref"], R)
    a1d = orc.ls_three_body(2, s_3pi, s_pipi, MPI, m_a1, g_a1, model["m_rho_ref"], R)
    k1a = orc.ls_three_body(0, s_kpipi, s_kpi, MPI, model["m_k1a"], model["g_k1a"],
                            model["m_ks_ref"], R)
    k1b = orc.ls_three_body(0, s_kpipi, s_kpi, MPI, model["m_k1b"], model["g_k1b"],
                            model["m_ks_ref"], R)
    fv = lambda L, q: orc.barrier(L, (R * q) ** 2)
    q_vv, q_a1, q_k1 = qd
    return np.array([
        sf[0] * ks * rho,
        sf[1] * fv(1, q_vv) * ks * rho,
        sf[2] * fv(2, q_vv) * ks * rho,
        sf[3] * fv(1, q_vv) * rho,
        sf[4] * fv(1, q_a1) * a1s * rho,
        sf[5] * fv(1, q_a1) * a1d * rho,
        sf[6] * fv(1, q_k1) * k1a * ks,
        sf[6] * fv(1, q_k1) * k1b * ks,
    ])


@pytest.fixture(scope="module")
def events():
    return I.phase_space(200, 23)


def _theta(model, seed, **shape):
    th = I.make_theta(model, I.draw_coefficients(model, seed))
    for k, v in shape.items():
        th[I.theta_index(model, k)] = v
    return th


def test_invariant_masses_and_d_vertex_momenta(orc, events):
    # the four invariants against four-vector sums, and the D-vertex momenta
    # against the Kallen function of those invariants
    for ev in events[:100]:
        _, qd, s = orc.spin_factors(ev, MD, MK, MPI)
        for sg in range(2):
            ref = invariants(ev, sg)
            assert np.allclose(s[sg], ref, rtol=1e-13, atol=0.0), (sg, s[sg], ref)
            s_kpi, s_pipi, s_kpipi, s_3pi = ref
            q_ref = [kallen_q(MD * MD, math.sqrt(s_kpi), math.sqrt(s_pipi)),
                     kallen_q(MD * MD, math.sqrt(s_3pi), MK),
                     kallen_q(MD * MD, math.sqrt(s_kpipi), MPI)]
            assert np.allclose(qd[sg], q_ref, rtol=1e-11, atol=1e-12)
        # s(3 pi) is the same in both configurations
        assert s[0][3] == s[1][3]


@pytest.mark.parametrize("model", [FULL, SMALL], ids=["fourteen", "four"])
@pytest.mark.parametrize("shape", [{}, dict(m_ks=0.91, g_ks=0.06, m_rho=0.76, g_rho=0.16,
                                            m_a1=1.26, g_a1=0.38)], ids=["nominal", "shifted"])
def test_basis_equals_chain_table(orc, events, model, shape):
    # B_k = b_k(a) + b_k(b) with b_k from the chain table, chain by chain
    th = _theta(model, 31, **shape)
    worst = 0.0
    for ev in events:
        B = orc.basis(model, th, ev)
        ref = chains(orc, model, th, ev, 0) + chains(orc, model, th, ev, 1)
        scale = np.abs(ref).max()
        for k in range(8):
            d = abs(B[k] - ref[k]) / scale
            worst = max(worst, d)
            assert d <= 1e-13, (k + 1, B[k], ref[k])
    assert worst <= 1e-13


def test_each_chain_differs_from_the_others(orc, events):
    # guard against a table in which two chains coincide: every pair of chains
    # must differ on these events (so a swapped chain cannot pass unnoticed)
    th = _theta(FULL, 31)
    B = np.array([orc.basis(FULL, th, ev) for ev in events[:50]])
    for k in range(8):
        for l in range(k + 1, 8):
            ratio = B[:, k] / B[:, l]
            assert np.ptp(ratio.real) + np.ptp(ratio.imag) > 1e-3, (k + 1, l + 1)


def test_bose_sum_is_plain_sum_of_configurations(orc, events):
    # the two configurations are exchanged by swapping the pi-: b_k(b) of an
    # event is b_k(a) of the swapped event, and B_k has no 1/sqrt(2)
    th = _theta(FULL, 37)
    for ev in events[:40]:
        sw = ev[[0, 3, 2, 1]]
        ba = chains(orc, FULL, th, ev, 0)
        bb = chains(orc, FULL, th, sw, 0)
        assert np.allclose(chains(orc, FULL, th, ev, 1), bb, rtol=1e-12, atol=0.0)
        assert np.allclose(orc.basis(FULL, th, ev), ba + bb, rtol=1e-13, atol=1e-13 * np.abs(ba + bb).max())


@pytest.mark.parametrize("model", [FULL, SMALL], ids=["fourteen", "four"])
def test_amplitude_membership(orc, events, model):
    # the presets carry the membership of the model description
    comp_a, comp_ab = MEMBERS[model["name"]]
    assert list(model["comp_a"]) == comp_a and list(model["comp_ab"]) == comp_ab
    na, nb = len(comp_a), len(comp_ab)
    base = _theta(model, 41)
    ev = events[:30]
    B = np.array([chains(orc, model, base, e, 0) + chains(orc, model, base, e, 1) for e in ev])

    def terms(ca, cb):
        th = base.copy()
        th[:2 * (na + nb)] = 0.0
        for j, c in ca:
            th[2 * j], th[2 * j + 1] = c.real, c.imag
        for j, c in cb:
            th[2 * (na + j)], th[2 * (na + j) + 1] = c.real, c.imag
        return orc.event_terms(model, th, ev.reshape(-1, 16))

    c1, c2 = 0.7 - 0.4j, -0.3 + 1.1j
    # one coefficient of A_f switched on: A = c B_k, Abar = 0
    for j, k in enumerate(comp_a):
        out = terms([(j, c1)], [])
        assert np.allclose(out[:, 0], abs(c1) ** 2 * np.abs(B[:, k - 1]) ** 2, rtol=1e-12, atol=0.0)
        assert np.all(out[:, 1] == 0.0)
    # one coefficient of Abar_f: Abar = c B_k, A = 0
    for j, k in enumerate(comp_ab):
        out = terms([], [(j, c2)])
        assert np.allclose(out[:, 1], abs(c2) ** 2 * np.abs(B[:, k - 1]) ** 2, rtol=1e-12, atol=0.0)
        assert np.all(out[:, 0] == 0.0)
    # one of each: the interference A Abar* = c1 B_k conj(c2 B_l)
    for j, k in enumerate(comp_a):
        for jb, kb in enumerate(comp_ab):
            out = terms([(j, c1)], [(jb, c2)])
            x = c1 * B[:, k - 1] * np.conj(c2 * B[:, kb - 1])
            tol = 1e-12 * np.abs(x).max()
            assert np.allclose(out[:, 2], x.real, rtol=0.0, atol=tol), (k, kb)
            assert np.allclose(out[:, 3], x.imag, rtol=0.0, atol=tol), (k, kb)
