"""CPU pins of the validation helpers (tests/two_sample.py): the five
projections recover the masses and angles of events built by explicit
two-body decays and boosts, are unchanged by rotating and boosting the whole
event, and the two-sample statistic is calibrated (uniform p-values for
samples of one density) and has power (small p-values otherwise)."""

import numpy as np

from two_sample import compare, projections

MD, MK, MPI = 1.86484, 0.493677, 0.13957


def _q(M, m1, m2):
    return np.sqrt((M * M - (m1 + m2) ** 2) * (M * M - (m1 - m2) ** 2)) / (2 * M)


def _lab(p, beta):
    """Boost four-vectors p [n,4] by velocity beta [n,3] (rest -> moving)."""
    b2 = np.sum(beta * beta, axis=1)
    g = 1.0 / np.sqrt(1.0 - b2)
    bp = np.sum(beta * p[:, 1:], axis=1)
    e = g * (p[:, 0] + bp)
    v = p[:, 1:] + ((g - 1.0) * bp / b2 + g * p[:, 0])[:, None] * beta
    return np.concatenate([e[:, None], v], axis=1)


def _build(m12, m34, c12, c34, phi):
    """Events with the given projections: in the D frame the 12 pair flies
    along +z and the 34 pair along -z; in the 12 rest frame the pi+ has polar
    angle acos(c12) to +z in the x-z plane; in the 34 rest frame the K+ has
    polar angle acos(c34) to -z at azimuth phi about the 12 direction."""
    n = len(m12)
    q = _q(MD, m12, m34)
    q12, q34 = _q(m12, MPI, MPI), _q(m34, MK, MPI)
    s12, s34 = np.sqrt(1 - c12 ** 2), np.sqrt(1 - c34 ** 2)
    d12 = np.stack([s12, np.zeros(n), c12], 1)
    # K+ direction in the 34 frame: polar angle to -z, azimuth phi measured
    # in the same right-handed sense about +z as the plane angle
    d34 = np.stack([s34 * np.cos(phi), s34 * np.sin(phi), -c34], 1)
    def pair(qv, d, ma, mb):
        pa = np.concatenate([np.sqrt(ma ** 2 + qv ** 2)[:, None], qv[:, None] * d], 1)
        pb = np.concatenate([np.sqrt(mb ** 2 + qv ** 2)[:, None], -qv[:, None] * d], 1)
        return pa, pb
    ppi, pam = pair(q12, d12, MPI, MPI)
    kp, pbm = pair(q34, d34, MK, MPI)
    b12 = np.stack([np.zeros(n), np.zeros(n), q / np.sqrt(q ** 2 + m12 ** 2)], 1)
    b34 = np.stack([np.zeros(n), np.zeros(n), -q / np.sqrt(q ** 2 + m34 ** 2)], 1)
    ppi, pam = _lab(ppi, b12), _lab(pam, b12)
    kp, pbm = _lab(kp, b34), _lab(pbm, b34)
    return np.stack([kp, pam, ppi, pbm], axis=1)


def _random_kinematics(rng, n):
    m12 = rng.uniform(2 * MPI + 0.01, 1.0, n)
    m34 = rng.uniform(MK + MPI + 0.01, MD - m12 - 0.01)
    return m12, m34, rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-np.pi, np.pi, n)


def test_projections_recover_constructed_events():
    rng = np.random.default_rng(1)
    m12, m34, c12, c34, phi = _random_kinematics(rng, 2000)
    p4 = _build(m12, m34, c12, c34, phi)
    pr = projections(p4)
    assert np.allclose(pr[:, 0], m12, atol=1e-12) and np.allclose(pr[:, 1], m34, atol=1e-12)
    assert np.allclose(pr[:, 2], c12, atol=1e-10) and np.allclose(pr[:, 3], c34, atol=1e-10)
    assert np.allclose(np.angle(np.exp(1j * (pr[:, 4] - phi))), 0.0, atol=1e-9)


def test_projections_are_frame_independent():
    rng = np.random.default_rng(2)
    p4 = _build(*_random_kinematics(rng, 500))
    # a random rotation, then a random boost of the whole event
    A = rng.normal(size=(3, 3))
    R, _ = np.linalg.qr(A)
    if np.linalg.det(R) < 0:
        R[:, 0] = -R[:, 0]
    q = p4.copy()
    q[..., 1:] = p4[..., 1:] @ R.T
    beta = np.tile(rng.uniform(-0.5, 0.5, 3), (len(q), 1))
    for i in range(4):
        q[:, i] = _lab(q[:, i], beta)
    a, b = projections(p4), projections(q)
    assert np.allclose(a[:, :4], b[:, :4], atol=1e-9)
    assert np.allclose(np.angle(np.exp(1j * (a[:, 4] - b[:, 4]))), 0.0, atol=1e-8)


def test_two_sample_statistic_is_calibrated_and_has_power():
    rng = np.random.default_rng(3)
    ps = []
    for _ in range(200):
        a = rng.normal(size=4000)
        b = rng.normal(size=6000)
        ps.append(compare(a, b, bins=20)[1])
    ps = np.array(ps)
    # uniform p-values: mean 1/2, and about 10% below 0.1
    assert abs(ps.mean() - 0.5) < 0.06
    assert 0.04 < np.mean(ps < 0.1) < 0.17
    # a 5% shift of the width is found
    a = rng.normal(size=50_000)
    b = 1.05 * rng.normal(size=50_000)
    assert compare(a, b)[1] < 1e-6
