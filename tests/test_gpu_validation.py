"""GPU: validation of generated pseudo-events by two-sample comparison of
the five phase-space projections m12, m34, cos12, cos34, phi and the decay
time (Sec. 3.2, where the comparison is against another framework's
generator; here against two generators written independently of the
library's kernels):

* the oracle's generator (counter-based, the same recipe in plain C++) with
  a different seed: an independent sample of the same density;
* the fixture generator (NumPy PCG64 GENBOD and accept-reject, the oracle's
  rate): an independent implementation of the sampling as well.

Each comparison passes when its chi^2 p-value is above 1e-3 and the bin
pulls have unit width; a comparison against uniform phase space must fail
(the test has power). The samples are seeded, so the outcome is fixed."""

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I
from two_sample import NAMES, compare, projections

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

MODEL = I.MODEL_FULL
MASSES = (MODEL["m_K"], MODEL["m_pi"], MODEL["m_pi"], MODEL["m_pi"])


@pytest.fixture(scope="module")
def samples(orc):
    from paper_1702_06735_amd import mixamp as M
    M.load_library()
    th = I.make_theta(MODEL, I.draw_coefficients(MODEL, 201))
    with M.Context(MODEL, device=0) as ctx:
        a4, at, st = ctx.draw_data(th, 500_000, seed=5001)
        u4, _, _, _ = ctx.generate(M.MXA_MC, 500_000, 5004)
        gpu = (a4.cpu().numpy().reshape(-1, 16), at.cpu().numpy())
        uni = u4.cpu().numpy().reshape(-1, 16)
    env = st["envelope"]
    wmax = I.genbod_wmax(MODEL["m_D"], MASSES)
    p4s, ts, first = [], [], 0
    while sum(len(t) for t in ts) < 500_000:
        need = 500_000 - sum(len(t) for t in ts)
        nc = int(need / 0.004) + 65536
        _, p4, t, s = orc.generate(MODEL, th, "data", 5003, nc, wmax, env, first=first, max_out=need)
        assert s[2] == 0, "envelope exceeded"
        p4s.append(p4.reshape(-1, 16))
        ts.append(t)
        first += nc
    ora = (np.concatenate(p4s), np.concatenate(ts))
    fn = lambda p, t: orc.event_terms(MODEL, th, p, t)
    d = I.draw_data(fn, 100_000, 5002, MODEL, th, n_env=200_000, batch=1 << 18)
    fix = (d.p4.reshape(-1, 16), d.t)
    return gpu, ora, fix, uni


def _table(x, y):
    px, py = projections(x[0]), projections(y[0])
    out = {}
    for i, name in enumerate(NAMES):
        out[name] = compare(px[:, i], py[:, i])
    if x[1] is not None and y[1] is not None:
        out["t"] = compare(x[1], y[1])
    return out


@pytest.mark.parametrize("other", ["oracle", "fixture"])
def test_generated_projections_agree(samples, other):
    gpu, ora, fix, _ = samples
    res = _table(gpu, ora if other == "oracle" else fix)
    for name, (c2, p, r) in res.items():
        print(f"gpu vs {other}: {name:6s} chi2/ndf {c2:6.1f}/{len(r) - 1}  p {p:.3f}  "
              f"pulls mean {r.mean():+.3f} width {r.std(ddof=1):.3f}", flush=True)
    for name, (c2, p, r) in res.items():
        assert p > 1e-3, (other, name, p)
        assert 0.75 < r.std(ddof=1) < 1.3, (other, name)


def test_comparison_has_power(samples):
    gpu, _, _, uni = samples
    res = _table(gpu, (uni, None))
    for name, (c2, p, r) in res.items():
        print(f"gpu vs uniform phase space: {name:6s} p {p:.2e}", flush=True)
    assert res["m12"][1] < 1e-10 and res["m34"][1] < 1e-10
