"""Pins of the oracle's break-up momentum, barrier factors and lineshapes.

Each check compares against something other than the oracle's own formula:
the rest-frame energy construction of the two-body momentum, spherical Hankel
functions for the Blatt-Weisskopf factors, the pole value and the Lorentzian
integral of a Breit-Wigner, and the threshold/asymptotic power laws of the
running width.
"""

import math

import numpy as np
import pytest
from scipy import integrate, special

from paper_1702_06735_amd import inputs as I

M = I.MODEL_FULL
MK, MPI, R = M["m_K"], M["m_pi"], M["r"]


def test_q2_matches_rest_frame_energy(orc):
    rng = np.random.default_rng(5)
    for _ in range(200):
        ma, mb = rng.uniform(0.05, 1.0, 2)
        Mt = (ma + mb) * rng.uniform(1.0001, 4.0)
        # in the rest frame of Mt: E_a = (M^2 + ma^2 - mb^2) / 2M, q^2 = E_a^2 - ma^2
        ea = (Mt * Mt + ma * ma - mb * mb) / (2.0 * Mt)
        ref = ea * ea - ma * ma
        assert orc.q2(Mt * Mt, ma, mb) == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_q2_clamped_below_threshold(orc):
    assert orc.q2(0.5 ** 2, 0.3, 0.3) == 0.0


def test_known_break_up_momenta(orc):
    # K*0 -> K pi at the K*0 mass and rho0 -> pi pi at the rho0 mass
    assert math.sqrt(orc.q2(0.8955 ** 2, MK, MPI)) == pytest.approx(0.290787, abs=2e-6)
    assert math.sqrt(orc.q2(0.7753 ** 2, MPI, MPI)) == pytest.approx(0.361653, abs=2e-6)


@pytest.mark.parametrize("L", [0, 1, 2])
def test_barrier_from_spherical_hankel(orc, L):
    # F_L(z)^-2 = z^L |x h_L(x)|^2 with x = sqrt(z) and h_L = j_L + i y_L
    for x in [0.05, 0.3, 0.9, 1.7, 3.2, 8.0]:
        z = x * x
        hh = special.spherical_jn(L, x) ** 2 + special.spherical_yn(L, x) ** 2
        ref = 1.0 / math.sqrt(z ** L * x * x * hh)
        assert orc.barrier(L, z) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("m0,g0,ma,mb", [(0.8955, 0.0473, MK, MPI), (0.7753, 0.1491, MPI, MPI)])
def test_two_body_pole_value(orc, m0, g0, ma, mb):
    # at s = m0^2: q = q0, B' = 1, Gamma(s) = Gamma0, LS = i / (m0 Gamma0)
    v = orc.ls_two_body(m0 * m0, m0, g0, ma, mb, R)
    assert abs(v.real) < 1e-12 * abs(v)
    assert v.imag == pytest.approx(1.0 / (m0 * g0), rel=1e-13)


def _width_and_barrier(orc, s, m0, g0, ma, mb):
    """Recover B'(s) and m0 Gamma(s) from the complex lineshape:
    1/LS = (m0^2 - s - i m0 Gamma(s)) / B'."""
    inv = 1.0 / orc.ls_two_body(s, m0, g0, ma, mb, R)
    bp = (m0 * m0 - s) / inv.real
    return bp, -inv.imag * bp


def test_two_body_running_width_power_laws(orc):
    m0, g0, ma, mb = 0.7753, 0.1491, MPI, MPI
    thr = (ma + mb) ** 2
    # near threshold m0 Gamma(s) ~ q^3: log-log slope in q tends to 3
    s1, s2 = thr * (1 + 1e-6), thr * (1 + 4e-6)
    q1, q2 = math.sqrt(orc.q2(s1, ma, mb)), math.sqrt(orc.q2(s2, ma, mb))
    w1 = _width_and_barrier(orc, s1, m0, g0, ma, mb)[1] * math.sqrt(s1)
    w2 = _width_and_barrier(orc, s2, m0, g0, ma, mb)[1] * math.sqrt(s2)
    assert math.log(w2 / w1) / math.log(q2 / q1) == pytest.approx(3.0, abs=1e-4)
    # far above, the barrier turns q^3 into q^1: sqrt(s) Gamma(s) / q -> const
    big = [1e7, 4e7]
    rat = [_width_and_barrier(orc, s, m0, g0, ma, mb)[1] * math.sqrt(s)
           / math.sqrt(orc.q2(s, ma, mb)) for s in big]
    assert rat[1] / rat[0] == pytest.approx(1.0, rel=1e-4)


def test_two_body_barrier_ratio(orc):
    # B'(s)^2 (1 + r^2 q^2) is constant in s (the F_1 ratio), equal to 1 + r^2 q0^2
    m0, g0 = 0.8955, 0.0473
    q0sq = orc.q2(m0 * m0, MK, MPI)
    for s in [0.45, 0.7, 0.9, 1.4, 1.9]:
        bp = _width_and_barrier(orc, s, m0, g0, MK, MPI)[0]
        assert bp * bp * (1 + R * R * orc.q2(s, MK, MPI)) == pytest.approx(
            1 + R * R * q0sq, rel=1e-12)


def test_constant_width_lorentzian_integral(orc):
    # int |1/(m0^2 - s - i m0 G0)|^2 ds over the real line = pi / (m0 G0)
    m0, g0 = 1.23, 0.42
    f = lambda s: abs(orc.ls_three_body(0, s, 0.6, MPI, m0, g0, 0.7753, R)) ** 2
    val, _ = integrate.quad(f, -np.inf, np.inf, epsabs=0, epsrel=1e-12, limit=400)
    assert val == pytest.approx(math.pi / (m0 * g0), rel=1e-10)


def test_three_body_d_wave_at_nominal_point(orc):
    # with the sub-resonance at its nominal mass and s = m0^2, B'_2 = 1
    m0, g0, mr = 1.23, 0.42, 0.7753
    v = orc.ls_three_body(2, m0 * m0, mr * mr, MPI, m0, g0, mr, R)
    assert abs(v.real) < 1e-13 * abs(v)
    assert v.imag == pytest.approx(1.0 / (m0 * g0), rel=1e-13)
    # away from it, |B'_2| follows the F_2 ratio built from the rest-frame momenta
    s, sr = 1.5, 0.5
    E = (s + sr - MPI ** 2) / (2 * math.sqrt(s))
    q2 = E * E - sr
    ea0 = (m0 * m0 + mr * mr - MPI ** 2) / (2 * m0)
    q02 = ea0 * ea0 - mr * mr
    ratio = math.sqrt((9 + 3 * R * R * q02 + (R * R * q02) ** 2)
                      / (9 + 3 * R * R * q2 + (R * R * q2) ** 2))
    v2 = orc.ls_three_body(2, s, sr, MPI, m0, g0, mr, R)
    v0 = orc.ls_three_body(0, s, sr, MPI, m0, g0, mr, R)
    assert abs(v2 / v0) == pytest.approx(ratio, rel=1e-12)
