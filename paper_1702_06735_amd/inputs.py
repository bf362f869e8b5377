"""Seeded synthetic inputs shared by the GPU library's callers and the oracle.

This module holds none of the likelihood's arithmetic. It provides
  * the model presets (resonance content and fixed constants) and workload
    configurations (sample sizes, seeds);
  * uniform four-body phase-space events by F. James' GENBOD method (CERN
    68-15, 1968), which is the role MCBooster plays in Sec. 3.1 of the paper;
  * decay times from exp(-Gamma t) cosh(y Gamma t), the envelope of the rate;
  * complex coefficients with |c| ~ U[0.5, 1.5], arg c ~ U[0, 2 pi);
  * an accept-reject loop that turns uniform events into pseudo-data
    (Sec. 3.1). The model's rate is passed in as a callable, so the loop
    itself evaluates nothing of the model.

Event layout: float64 ``[n, 4, 4]`` in the order K+, pi-(a), pi+, pi-(b), each
(E, px, py, pz) in GeV in the D0 rest frame; decay times float64 ``[n]`` in ps.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Model presets. Basis index k: 1 K*0 rho0 S, 2 K*0 rho0 P, 3 K*0 rho0 D,
# 4 (K+pi-)_S rho0, 5 a1 -> rho pi S, 6 a1 -> rho pi D, 7 K1(1270) -> K* pi,
# 8 K1(1400) -> K* pi.
# ---------------------------------------------------------------------------
_CONST = dict(
    m_D=1.86484, m_K=0.493677, m_pi=0.13957,
    tau=0.4101,            # D0 lifetime [ps], Gamma = 1/tau
    r=1.5,                 # Blatt-Weisskopf radius [1/GeV] at every vertex
    m_ks_ref=0.8955, m_rho_ref=0.7753,
    m_k1a=1.272, g_k1a=0.09,
    m_k1b=1.403, g_k1b=0.174,
)
_FLOAT0 = dict(x=0.0049, y=0.0061, m_ks=0.8955, g_ks=0.0473, m_rho=0.7753, g_rho=0.1491,
               m_a1=1.23, g_a1=0.42)

#: A_f = K*0 rho0 S-wave + (K+pi-)_S rho0; Abar_f = a1 -> rho pi (with K+) + K*0 rho0 P-wave
MODEL_SMALL = dict(_CONST, **_FLOAT0, name="four-component", comp_a=[1, 4], comp_ab=[5, 2])
#: A_f with 6 components, Abar_f with 8
MODEL_FULL = dict(_CONST, **_FLOAT0, name="fourteen-component",
                  comp_a=[1, 2, 3, 4, 7, 8], comp_ab=[1, 2, 3, 4, 5, 6, 7, 8])


def with_background(model: dict, g_bkg: float = 1.0 / 0.8, f_bkg: float = 0.1) -> dict:
    """The model with a background component: events uniform in phase space
    with decay times from Gamma_b exp(-Gamma_b t) (Gamma_b = ``g_bkg`` [1/ps];
    the default is a lifetime of 0.8 ps), fraction ``f_bkg`` of the data (an
    extra, last parameter)."""
    return dict(model, name=model["name"] + " + background", g_bkg=float(g_bkg),
                f_bkg=float(f_bkg))


def with_cp_violation(model: dict, qp_abs: float = 1.0, qp_arg: float = 0.0) -> dict:
    """The model with CP violation in mixing: q/p = qp_abs exp(i qp_arg) is
    free (two extra, last parameters) and the data carry flavour tags."""
    return dict(model, name=model["name"] + " + CP violation", cpv=True, qp_abs=float(qp_abs),
                qp_arg=float(qp_arg))


def with_resolution(model: dict, sigma_t: float = 0.06) -> dict:
    """The model with a Gaussian decay-time resolution of width ``sigma_t``
    [ps] (a fixed constant, no extra parameter)."""
    return dict(model, name=model["name"] + " + resolution", sigma_t=float(sigma_t))


def cp_conjugate(p4):
    """CP conjugate of events [n,4,4]: 3-momenta negated (parity); with the
    charge conjugation the particle slots K+, pi-, pi+, pi- hold K-, pi+, pi-,
    pi+ and vice versa, so the slot order is kept."""
    out = np.array(p4, dtype=np.float64, copy=True).reshape(-1, 4, 4)
    out[..., 1:] = -out[..., 1:]
    return out


@dataclass(frozen=True)
class Workload:
    name: str
    model: dict
    n_data: int
    n_mc: int
    seed_coeff: int
    seed_mc: int
    seed_data: int
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    # four-component model, 10k data / 100k MC (small case the oracle finishes in seconds)
    "small": Workload("small", MODEL_SMALL, 10_000, 100_000, 101, 102, 103),
    # fourteen-component model, 50k data / 4M MC (the headline evaluation)
    "full": Workload("full", MODEL_FULL, 50_000, 4_000_000, 201, 202, 203),
    # precision form: 10M data / 50M MC
    "precision": Workload("precision", MODEL_FULL, 10_000_000, 50_000_000, 301, 302, 303),
    # differentiation form: 1M data / 4M MC
    "gradient": Workload("gradient", MODEL_FULL, 1_000_000, 4_000_000, 401, 402, 403),
    # serving form: 512 pseudo-experiment fits sharing a 4M MC sample
    "serving": Workload("serving", MODEL_FULL, 0, 4_000_000, 501, 502, 503,
                        extra=dict(n_fits=512, n_min=5_000, n_max=500_000, jitter=0.002,
                                   rate_hz=200.0, seed_sizes=504, seed_arrivals=505)),
}

FLOAT_NAMES = ("x", "y", "m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1")


def has_background(model: dict) -> bool:
    return float(model.get("g_bkg", 0.0)) > 0.0


def float_names(model: dict) -> tuple:
    extra = (("qp_abs", "qp_arg") if model.get("cpv") else ()) + \
        (("f_bkg",) if has_background(model) else ())
    return FLOAT_NAMES + extra


def n_theta(model: dict) -> int:
    return 2 * (len(model["comp_a"]) + len(model["comp_ab"])) + len(float_names(model))


def draw_coefficients(model: dict, seed: int) -> np.ndarray:
    """Complex coefficients of A_f then Abar_f members: |c| ~ U[0.5,1.5], arg ~ U[0,2pi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(model["comp_a"]) + len(model["comp_ab"])
    out = np.empty(n, dtype=np.complex128)
    for i in range(n):
        mag = rng.uniform(0.5, 1.5)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        out[i] = mag * complex(math.cos(ph), math.sin(ph))
    return out


def make_theta(model: dict, coeffs: np.ndarray, **overrides) -> np.ndarray:
    """Parameter vector: (Re, Im) of A_f then Abar_f coefficients, x, y, and
    mass and width of K*0, rho0 and a1(1260)."""
    c = np.asarray(coeffs, dtype=np.complex128)
    assert c.size == len(model["comp_a"]) + len(model["comp_ab"])
    names = float_names(model)
    vals = dict((k, model[k]) for k in names)
    vals.update(overrides)
    th = np.empty(n_theta(model))
    th[0:2 * c.size:2] = c.real
    th[1:2 * c.size:2] = c.imag
    th[2 * c.size:] = [vals[k] for k in names]
    return th


def theta_index(model: dict, name: str) -> int:
    return 2 * (len(model["comp_a"]) + len(model["comp_ab"])) + float_names(model).index(name)


# ---------------------------------------------------------------------------
# Uniform four-body phase space (GENBOD)
# ---------------------------------------------------------------------------

def _pstar(M, m1, m2):
    """Momentum of either daughter in the rest frame of a mass-M system."""
    a = (M * M - (m1 + m2) ** 2) * (M * M - (m1 - m2) ** 2)
    return np.sqrt(np.maximum(a, 0.0)) / (2.0 * M)


def _isotropic(rng, n):
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], axis=1)


def _boost(p, P, M):
    """Boost four-vectors ``p`` [n,4] from the rest frame of a system with mass
    ``M`` [n] to the frame where it has four-momentum ``P`` [n,4]."""
    E = p[:, 0]
    pdot = np.einsum("ij,ij->i", p[:, 1:], P[:, 1:])
    E2 = (E * P[:, 0] + pdot) / M
    f = (E + E2) / (P[:, 0] + M)
    out = np.empty_like(p)
    out[:, 0] = E2
    out[:, 1:] = p[:, 1:] + f[:, None] * P[:, 1:]
    return out


def _two_body(q, n_hat, ma, mb):
    """Back-to-back pair with momentum q along n_hat in its rest frame."""
    pa = np.empty((q.size, 4))
    pb = np.empty((q.size, 4))
    pa[:, 0] = np.sqrt(q * q + ma * ma)
    pb[:, 0] = np.sqrt(q * q + mb * mb)
    pa[:, 1:] = q[:, None] * n_hat
    pb[:, 1:] = -q[:, None] * n_hat
    return pa, pb


def genbod_weights(M, masses, r):
    """GENBOD weight of each candidate.

    ``r`` [n,2] are sorted uniforms. Intermediate masses
    M2 = m0+m1 + r0 T, M3 = m0+m1+m2 + r1 T, T = M - sum(m); the weight is the
    product of the break-up momenta q(M2; m0, m1) q(M3; M2, m2) q(M; M3, m3).
    """
    m0, m1, m2, m3 = masses
    T = M - sum(masses)
    M2 = m0 + m1 + r[:, 0] * T
    M3 = m0 + m1 + m2 + r[:, 1] * T
    q2 = _pstar(M2, m0, m1)
    q3 = _pstar(M3, M2, m2)
    q4 = _pstar(np.full_like(M3, M), M3, m3)
    return q2 * q3 * q4, (M2, M3, q2, q3, q4)


_WMAX = {}


def genbod_wmax(M, masses):
    """Upper bound of the GENBOD weight: 1.01 x its maximum over a 1001 x 1001
    grid of (r0 <= r1). The weight is smooth, so the grid maximum is within
    ~1e-6 of the true one; the textbook bound (each q at its own extreme) is
    valid too but ~9x looser for this final state."""
    key = (float(M),) + tuple(float(m) for m in masses)
    if key not in _WMAX:
        g = np.linspace(0.0, 1.0, 1001)
        r0, r1 = np.meshgrid(g, g, indexing="ij")
        sel = r0 <= r1
        w, _ = genbod_weights(M, masses, np.stack([r0[sel], r1[sel]], axis=1))
        _WMAX[key] = 1.01 * float(w.max())
    return _WMAX[key]


def phase_space(n, rng, M=None, masses=None, batch=1 << 20):
    """``n`` events uniform in four-body phase space, ``[n,4,4]`` float64.

    ``rng`` is a seed or a ``numpy.random.Generator`` (PCG64). Each candidate
    draws, in order: two uniforms for the intermediate masses, one for
    acceptance, and three isotropic directions.
    """
    if not isinstance(rng, np.random.Generator):
        rng = np.random.Generator(np.random.PCG64(rng))
    if M is None:
        M = _CONST["m_D"]
    if masses is None:
        masses = (_CONST["m_K"], _CONST["m_pi"], _CONST["m_pi"], _CONST["m_pi"])
    m0, m1, m2, m3 = masses
    wmax = genbod_wmax(M, masses)
    out = np.empty((n, 4, 4))
    filled = 0
    while filled < n:
        nb = batch
        r = np.sort(rng.random((nb, 2)), axis=1)
        u = rng.random(nb)
        d2 = _isotropic(rng, nb)
        d3 = _isotropic(rng, nb)
        d4 = _isotropic(rng, nb)
        w, (M2, M3, q2, q3, q4) = genbod_weights(M, masses, r)
        acc = u * wmax < w
        k = min(int(acc.sum()), n - filled)
        idx = np.nonzero(acc)[0][:k]
        M2, M3, q2, q3, q4 = M2[idx], M3[idx], q2[idx], q3[idx], q4[idx]
        # (0 1) in the rest frame of M2
        p0, p1 = _two_body(q2, d2[idx], m0, m1)
        # (01) 2 in the rest frame of M3
        P01, p2 = _two_body(q3, d3[idx], M2, m2)
        p0 = _boost(p0, P01, M2)
        p1 = _boost(p1, P01, M2)
        # (012) 3 in the rest frame of M
        P012, p3 = _two_body(q4, d4[idx], M3, m3)
        p0 = _boost(p0, P012, M3)
        p1 = _boost(p1, P012, M3)
        p2 = _boost(p2, P012, M3)
        out[filled:filled + k, 0] = p0
        out[filled:filled + k, 1] = p1
        out[filled:filled + k, 2] = p2
        out[filled:filled + k, 3] = p3
        filled += k
    return out


def decay_times(rng, n, gamma, y):
    """Times from exp(-Gamma t) cosh(y Gamma t): a two-exponential mixture with
    rate Gamma(1-y) (probability (1+y)/2) or Gamma(1+y)."""
    pick = rng.random(n) < 0.5 * (1.0 + y)
    lam = np.where(pick, gamma * (1.0 - y), gamma * (1.0 + y))
    return rng.standard_exponential(n) / lam


def background_events(n, seed, g_bkg):
    """``n`` background events: uniform in phase space, decay times from
    Gamma_b exp(-Gamma_b t). Returns (p4 [n,4,4], t [n])."""
    rng = np.random.Generator(np.random.PCG64([seed, 3]))
    p4 = phase_space(n, rng)
    return p4, rng.standard_exponential(n) / float(g_bkg)


@dataclass
class DataSample:
    p4: np.ndarray
    t: np.ndarray
    envelope: float
    n_candidates: int
    exceedances: int


def draw_data(terms_fn, n, seed, model, theta, n_env=1_000_000, batch=1 << 18,
              safety=1.2):
    """Pseudo-data by accept-reject (Sec. 3.1): uniform phase-space candidates
    with decay times from the cosh envelope, kept with probability
    B / (2 cosh(y Gamma t) M_Phi).

    ``terms_fn(p4, t)`` returns per-event ``[m, 5]`` columns |A|^2, |Abar|^2,
    Re(A Abar*), Im(A Abar*), rate (Eq. (1) at t). ``M_Phi`` is ``safety``
    times the largest |A|^2 + |Abar|^2 over ``n_env`` uniform events, so that
    B <= 2 cosh(y Gamma t)(|A|^2+|Abar|^2) <= 2 cosh(y Gamma t) M_Phi. A
    candidate above the envelope restarts the draw with a 1.5x larger M_Phi.
    """
    y = float(theta[theta_index(model, "y")])
    gamma = 1.0 / model["tau"]
    env_rng = np.random.Generator(np.random.PCG64([seed, 1]))
    env = phase_space(n_env, env_rng)
    te = terms_fn(env, None)
    m_phi = safety * float(np.max(te[:, 0] + te[:, 1]))
    del env, te
    while True:
        rng = np.random.Generator(np.random.PCG64([seed, 2]))
        keep_p, keep_t = [], []
        got = ncand = exceed = 0
        while got < n:
            p4 = phase_space(batch, rng)
            t = decay_times(rng, batch, gamma, y)
            u = rng.random(batch)
            te = terms_fn(p4, t)
            ncand += batch
            exceed += int(np.count_nonzero(te[:, 0] + te[:, 1] > m_phi))
            if exceed:
                break
            acc = u * (2.0 * np.cosh(y * gamma * t) * m_phi) < te[:, 4]
            k = min(int(acc.sum()), n - got)
            idx = np.nonzero(acc)[0][:k]
            keep_p.append(p4[idx])
            keep_t.append(t[idx])
            got += k
        if exceed:
            m_phi *= 1.5
            continue
        return DataSample(np.concatenate(keep_p), np.concatenate(keep_t), m_phi, ncand, 0)


def swap_pions(p4):
    """The same events with the two pi- exchanged (Bose partner)."""
    out = np.array(p4, copy=True)
    out[:, [1, 3]] = out[:, [3, 1]]
    return out
