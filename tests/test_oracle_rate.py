"""Pins of the oracle's time-dependent rate, Eq. (1), and its time integral.

* Limits: x = y = 0 gives 2|A|^2; A = 0 and Abar = 0 leave single terms.
* The mixing identity: with q/p = 1, x = (m1 - m2)/Gamma and
  y = (Gamma1 - Gamma2)/(2 Gamma), the rate equals
  2 e^{Gamma t} |g+ A + g- Abar|^2 with g+- = (e^{-i l1 t} +- e^{-i l2 t})/2,
  l_k = m_k - i Gamma_k / 2. This fixes every sign of the interference terms.
* The closed-form time integral against adaptive quadrature.
"""

import cmath
import math

import numpy as np
import pytest
from scipy import integrate

G = 1.0 / 0.4101


def _rand_amp(rng):
    return complex(*rng.normal(size=2)) * rng.uniform(0.2, 3.0)


def test_no_mixing_limit(orc):
    rng = np.random.default_rng(1)
    for _ in range(50):
        A, Ab = _rand_amp(rng), _rand_amp(rng)
        t = rng.exponential(1 / G)
        assert orc.rate(A, Ab, 0.0, 0.0, G, t) == pytest.approx(2 * abs(A) ** 2, rel=1e-14)
        assert orc.rate_integrated(A, Ab, 0.0, 0.0, G) == pytest.approx(
            2 * abs(A) ** 2 / G, rel=1e-14)


def test_single_amplitude_limits(orc):
    rng = np.random.default_rng(2)
    for _ in range(50):
        A = _rand_amp(rng)
        x, y = rng.uniform(-0.05, 0.05, 2)
        t = rng.exponential(3 / G)
        cy, cx = math.cosh(y * G * t), math.cos(x * G * t)
        assert orc.rate(0j, A, x, y, G, t) == pytest.approx(abs(A) ** 2 * (cy - cx), rel=1e-9,
                                                           abs=1e-15)
        assert orc.rate(A, 0j, x, y, G, t) == pytest.approx(abs(A) ** 2 * (cy + cx), rel=1e-14)


def test_mixing_identity_fixes_signs(orc):
    rng = np.random.default_rng(3)
    for _ in range(200):
        A, Ab = _rand_amp(rng), _rand_amp(rng)
        x, y = rng.uniform(-0.3, 0.3, 2)
        t = rng.exponential(2 / G)
        # two mass eigenstates with mean width G
        m2 = 1.86
        m1 = m2 + x * G
        g1, g2 = G * (1 + y), G * (1 - y)
        l1, l2 = m1 - 0.5j * g1, m2 - 0.5j * g2
        gp = 0.5 * (cmath.exp(-1j * l1 * t) + cmath.exp(-1j * l2 * t))
        gm = 0.5 * (cmath.exp(-1j * l1 * t) - cmath.exp(-1j * l2 * t))
        ref = 2.0 * math.exp(G * t) * abs(gp * A + gm * Ab) ** 2
        assert orc.rate(A, Ab, x, y, G, t) == pytest.approx(ref, rel=1e-11)
        assert orc.rate(A, Ab, x, y, G, t) >= 0.0


def test_time_integral_against_quadrature(orc):
    rng = np.random.default_rng(4)
    for _ in range(30):
        A, Ab = _rand_amp(rng), _rand_amp(rng)
        x, y = rng.uniform(-0.5, 0.5, 2)
        f = lambda t: math.exp(-G * t) * orc.rate(A, Ab, x, y, G, t)
        # the integrand falls as exp(-G (1 - |y|) t); beyond 80 such lifetimes it is < 1e-34
        tmax = 80.0 / (G * (1.0 - abs(y)))
        val, _ = integrate.quad(f, 0.0, tmax, epsabs=0, epsrel=1e-13, limit=400)
        assert orc.rate_integrated(A, Ab, x, y, G) == pytest.approx(val, rel=1e-11)
