"""Distribution checks of uniform four-body phase-space samples, shared by the
tests of the fixture generator, the oracle's generator and the GPU generator."""

import math

import numpy as np
from scipy import stats


def msq(p):
    return p[..., 0] ** 2 - (p[..., 1:] ** 2).sum(-1)


def breakup(M, a, b):
    v = (M * M - (a + b) ** 2) * (M * M - (a - b) ** 2)
    return np.sqrt(np.clip(v, 0, None)) / (2 * M)


def constraint_error(ev, m_D, masses):
    """Largest violation of four-momentum conservation and of the mass shells."""
    tot = ev.sum(axis=1)
    return max(np.abs(tot[:, 0] - m_D).max(), np.abs(tot[:, 1:]).max(),
               np.abs(msq(ev) - np.asarray(masses) ** 2).max())


def pair_mass_pvalue(ev, m_D, m_K, m_pi, nb=16, sub=24):
    """chi^2 p-value of the (m(K+ pi-a), m(pi+ pi-b)) histogram against the
    phase-space density q(M; m1, m2) q(m1; m_K, m_pi) q(m2; m_pi, m_pi)."""
    m1 = np.sqrt(msq(ev[:, 0] + ev[:, 1]))
    m2 = np.sqrt(msq(ev[:, 2] + ev[:, 3]))
    e1 = np.linspace(m_K + m_pi, m_D - 2 * m_pi, nb + 1)
    e2 = np.linspace(2 * m_pi, m_D - m_K - m_pi, nb + 1)
    obs, _, _ = np.histogram2d(m1, m2, bins=[e1, e2])
    exp = np.zeros((nb, nb))
    for i in range(nb):
        a = e1[i] + (np.arange(sub) + 0.5) * (e1[i + 1] - e1[i]) / sub
        for j in range(nb):
            b = e2[j] + (np.arange(sub) + 0.5) * (e2[j + 1] - e2[j]) / sub
            A, B = np.meshgrid(a, b, indexing="ij")
            dens = breakup(m_D, A, B) * breakup(A, m_K, m_pi) * breakup(B, m_pi, m_pi)
            dens[A + B >= m_D] = 0.0
            exp[i, j] = dens.mean()
    exp *= obs.sum() / exp.sum()
    sel = exp > 20
    chi2 = np.sum((obs[sel] - exp[sel]) ** 2 / exp[sel])
    return stats.chi2.sf(chi2, sel.sum() - 1)


def isotropy_ok(ev, k=0, nsig=5.0):
    """Particle k's direction in the D rest frame: <cos> = 0, <cos^2> = 1/3."""
    c = ev[:, k, 3] / np.linalg.norm(ev[:, k, 1:], axis=1)
    n = len(c)
    return (abs(c.mean()) < nsig * math.sqrt(1 / 3 / n)
            and abs((c ** 2).mean() - 1 / 3) < nsig * math.sqrt(4 / 45 / n))
