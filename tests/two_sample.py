"""Phase-space projections of D0 -> K+ pi- pi+ pi- events and a binned
two-sample comparison (test infrastructure).

Sec. 3.2 (validation) compares generated samples in five variables: m12 and
m34, the invariant masses of the pi+ pi- pair (12) and of the K+ pi- pair
(34); cos12 and cos34, the helicity angles of the pi+ in the 12 rest frame
and of the K+ in the 34 rest frame, each measured from the pair's flight
direction in the D0 rest frame; and phi, the angle between the two decay
planes in the D0 rest frame. Particle order of an event: K+, pi-(a), pi+,
pi-(b); the 12 pair is (pi+, pi-(a)) and the 34 pair (K+, pi-(b)). (The
model is Bose-symmetric in the two pi-, so either pairing is a valid choice
as long as both samples use the same one.)
"""

import numpy as np


def _dot4(a, b):
    return a[..., 0] * b[..., 0] - np.sum(a[..., 1:] * b[..., 1:], axis=-1)


def boost_to_rest(p, P):
    """Four-vectors p [n,4] in the rest frame of P [n,4] (pure boost)."""
    M = np.sqrt(_dot4(P, P))
    b = P[:, 1:] / P[:, :1]
    b2 = np.sum(b * b, axis=1)
    g = P[:, 0] / M
    bp = np.sum(b * p[:, 1:], axis=1)
    gg = np.where(b2 > 0, (g - 1.0) / np.where(b2 > 0, b2, 1.0), 0.0)
    e = g * (p[:, 0] - bp)
    v = p[:, 1:] + (gg * bp - g * p[:, 0])[:, None] * b
    return np.concatenate([e[:, None], v], axis=1)


def _unit(v):
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def projections(p4):
    """[n,5]: m12, m34, cos12, cos34, phi (radians, in (-pi, pi])."""
    p4 = np.asarray(p4, dtype=np.float64).reshape(-1, 4, 4)
    D = p4.sum(axis=1)
    k, pa, pp, pb = (boost_to_rest(p4[:, i], D) for i in range(4))
    P12, P34 = pp + pa, k + pb
    m12 = np.sqrt(_dot4(P12, P12))
    m34 = np.sqrt(_dot4(P34, P34))
    z12 = _unit(P12[:, 1:])
    z34 = _unit(P34[:, 1:])
    cos12 = np.sum(_unit(boost_to_rest(pp, P12)[:, 1:]) * z12, axis=1)
    cos34 = np.sum(_unit(boost_to_rest(k, P34)[:, 1:]) * z34, axis=1)
    # decay planes in the D frame, oriented so that phi = 0 when the pi+ and
    # the K+ lie on the same side of the common axis
    n12 = _unit(np.cross(pp[:, 1:], pa[:, 1:]))
    n34 = _unit(np.cross(pb[:, 1:], k[:, 1:]))
    cphi = np.sum(n12 * n34, axis=1)
    sphi = np.sum(np.cross(n12, n34) * z12, axis=1)
    return np.stack([m12, m34, cos12, cos34, np.arctan2(sphi, cphi)], axis=1)


NAMES = ("m12", "m34", "cos12", "cos34", "phi")


def compare(a, b, bins=50):
    """Binned two-sample chi^2 of 1-d samples a and b: equal-population bins
    of the pooled sample; per bin the normalised difference
    r_i = (n_a sqrt(N_b/N_a) - n_b sqrt(N_a/N_b)) / sqrt(n_a + n_b), which is
    unit normal when both samples come from one density; chi^2 = sum r_i^2
    with bins - 1 degrees of freedom. Returns (chi2, p-value, pulls)."""
    from scipy.stats import chi2 as chi2_dist
    a = np.asarray(a)
    b = np.asarray(b)
    edges = np.quantile(np.concatenate([a, b]), np.linspace(0.0, 1.0, bins + 1))
    edges[0], edges[-1] = -np.inf, np.inf
    na = np.histogram(a, edges)[0].astype(np.float64)
    nb = np.histogram(b, edges)[0].astype(np.float64)
    ka, kb = np.sqrt(len(b) / len(a)), np.sqrt(len(a) / len(b))
    r = (na * ka - nb * kb) / np.sqrt(na + nb)
    c2 = float(np.sum(r * r))
    return c2, float(chi2_dist.sf(c2, bins - 1)), r
