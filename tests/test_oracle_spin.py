"""Pins of the oracle's covariant spin factors (Sec. 3, Fig. 2 topologies).

The oracle builds the orbital tensors by projection in Minkowski space. Here
the same quantities are rebuilt by explicit Lorentz boosts into each
resonance rest frame, where the rank-1 tensor of a vertex P -> u v is
(0, u* - v*) and the rank-2 tensor is the traceless symmetric product of
3-vectors. That is an independent arithmetic route, so a wrong operand, index
or sign in either fails. Further pins: Lorentz and rotation invariance, parity
(only the P-wave factor flips), and vanishing P-wave for coplanar events.
"""

import math

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

M = I.MODEL_FULL
MD, MK, MPI = M["m_D"], M["m_K"], M["m_pi"]


def mdot(a, b):
    return a[0] * b[0] - a[1:] @ b[1:]


def to_rest(p, P):
    """Components of p in the rest frame of P (pure boost)."""
    m = math.sqrt(mdot(P, P))
    e = (p[0] * P[0] - p[1:] @ P[1:]) / m
    f = (p[0] + e) / (P[0] + m)
    return np.concatenate([[e], p[1:] - f * P[1:]])


def from_rest(p, P):
    """Inverse of to_rest: components in the frame where the system has P."""
    m = math.sqrt(mdot(P, P))
    e = (p[0] * P[0] + p[1:] @ P[1:]) / m
    f = (p[0] + e) / (P[0] + m)
    return np.concatenate([[e], p[1:] + f * P[1:]])


def rel_vec(P, u, v):
    """Rank-1 orbital tensor of P -> u v: (0, u* - v*) in the P rest frame, boosted back."""
    us, vs = to_rest(u, P), to_rest(v, P)
    return from_rest(np.concatenate([[0.0], us[1:] - vs[1:]]), P)


def spatial_in(P, a):
    return to_rest(a, P)[1:]


def helicity_spin_factors(ev, sigma):
    p = [np.asarray(ev[i], dtype=float) for i in range(4)]
    k, pip = p[0], p[2]
    ps, po = (p[1], p[3]) if sigma == 0 else (p[3], p[1])
    pD = k + pip + ps + po
    P1, P2 = k + ps, pip + po
    t1, t2 = rel_vec(P1, k, ps), rel_vec(P2, pip, po)
    lD = rel_vec(pD, P1, P2)
    # 3-vectors in the D rest frame
    t1d, t2d, ld = spatial_in(pD, t1), spatial_in(pD, t2), spatial_in(pD, lD)
    md = math.sqrt(mdot(pD, pD))
    sf_s = mdot(t1, t2)
    sf_p = -md * ld @ np.cross(t1d, t2d)
    sf_d = (t1d @ ld) * (t2d @ ld) - (ld @ ld) * (t1d @ t2d) / 3.0
    sv = -(ld @ t2d)
    # a1 chain, 3-vectors in the a1 rest frame
    PA = pip + ps + po
    tV = rel_vec(P2, pip, po)
    lDa = rel_vec(pD, PA, k)
    lA = spatial_in(PA, P2) - spatial_in(PA, ps)
    la, ta = spatial_in(PA, lDa), spatial_in(PA, tV)
    a1s = -(la @ ta)
    a1d = (la @ lA) * (ta @ lA) - (lA @ lA) * (la @ ta) / 3.0
    # K1 chain, 3-vectors in the K1 rest frame
    PK = k + ps + pip
    tK = rel_vec(P1, k, ps)
    lDk = rel_vec(pD, PK, po)
    k1 = -(spatial_in(PK, lDk) @ spatial_in(PK, tK))
    # D-vertex momenta: |3-momentum| of one system in the D rest frame
    qvv = np.linalg.norm(spatial_in(pD, P1))
    qa1 = np.linalg.norm(spatial_in(pD, PA))
    qk1 = np.linalg.norm(spatial_in(pD, PK))
    return np.array([sf_s, sf_p, sf_d, sv, a1s, a1d, k1]), np.array([qvv, qa1, qk1])


@pytest.fixture(scope="module")
def events():
    return I.phase_space(300, 11)


def test_spin_factors_match_rest_frame_construction(orc, events):
    for ev in events:
        sf, qd, _ = orc.spin_factors(ev, MD, MK, MPI)
        for sg in range(2):
            ref_sf, ref_q = helicity_spin_factors(ev, sg)
            # the typical size of a factor sets the floor for ones that cancel
            typ = np.abs(ref_sf).max()
            assert np.all(np.abs(sf[sg] - ref_sf) <= 1e-10 * typ), (sg, sf[sg], ref_sf)
            assert np.allclose(qd[sg], ref_q, rtol=1e-12, atol=1e-11)


def _boost_event(ev, beta):
    b = np.asarray(beta)
    g = 1.0 / math.sqrt(1.0 - b @ b)
    out = np.empty_like(ev)
    for i, p in enumerate(ev):
        bp = b @ p[1:]
        out[i, 0] = g * (p[0] + bp)
        out[i, 1:] = p[1:] + ((g - 1.0) * bp / (b @ b) + g * p[0]) * b
    return out


def _rot(ev, R):
    out = np.array(ev, copy=True)
    out[:, 1:] = ev[:, 1:] @ R.T
    return out


def test_lorentz_and_rotation_invariance(orc, events):
    rng = np.random.default_rng(3)
    for ev in events[:60]:
        ref, _, _ = orc.spin_factors(ev, MD, MK, MPI)
        typ = np.abs(ref).max()
        gamma = rng.uniform(1.0, 10.0)
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        beta = n * math.sqrt(1.0 - 1.0 / gamma ** 2)
        b, _, _ = orc.spin_factors(_boost_event(ev, beta), MD, MK, MPI)
        assert np.all(np.abs(b - ref) <= 1e-9 * typ)
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        r, _, _ = orc.spin_factors(_rot(ev, q), MD, MK, MPI)
        assert np.all(np.abs(r - ref) <= 1e-12 * typ)


def test_parity_flips_only_p_wave(orc, events):
    for ev in events[:60]:
        ref, _, _ = orc.spin_factors(ev, MD, MK, MPI)
        flipped = np.array(ev, copy=True)
        flipped[:, 1:] *= -1.0
        f, _, _ = orc.spin_factors(flipped, MD, MK, MPI)
        typ = np.abs(ref).max()
        sign = np.ones(7)
        sign[1] = -1.0
        assert np.all(np.abs(f - sign * ref) <= 1e-13 * typ)


def test_coplanar_event_has_no_p_wave(orc, events):
    for ev in events[:40]:
        # flatten every momentum into the x-y plane with on-shell energies and
        # balance the 3-momentum with the pi+ (energy conservation is not
        # needed for the triple product to vanish)
        flat = np.array(ev, copy=True)
        flat[:, 3] = 0.0
        flat[:, 0] = np.sqrt(np.array([MK, MPI, MPI, MPI]) ** 2 + (flat[:, 1:] ** 2).sum(1))
        flat[2, 1:] = -(flat[0, 1:] + flat[1, 1:] + flat[3, 1:])
        flat[2, 0] = math.sqrt(MPI ** 2 + flat[2, 1:] @ flat[2, 1:])
        sf, _, _ = orc.spin_factors(flat, MD, MK, MPI)
        typ = np.abs(sf).max()
        assert np.all(np.abs(sf[:, 1]) <= 1e-13 * typ)


def test_orbital_tensor_orthogonality_and_norm(events):
    # the rank-1 tensor used above is orthogonal to P with t.t = -4 q*^2
    for ev in events[:20]:
        k, pa = ev[0], ev[1]
        P = k + pa
        t = rel_vec(P, k, pa)
        assert abs(mdot(t, P)) < 1e-13
        s = mdot(P, P)
        ea = (s + MK ** 2 - MPI ** 2) / (2 * math.sqrt(s))
        assert mdot(t, t) == pytest.approx(-4.0 * (ea * ea - MK ** 2), rel=1e-12)
