"""Host build of the library's decay-time resolution functions
(csrc/resolution.h): the Faddeeva function by Weideman's series against
SciPy's implementation, and the convolved exponential E(a; t) and its a
derivative against the closed form erfc expression and central differences."""

import os
import subprocess

import numpy as np
import pytest
from scipy.special import wofz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = r'''
#include <cstdio>
#include "resolution.h"
int main() {
  char mode;
  double a, b, c, d;
  while (std::scanf(" %c %lf %lf %lf %lf", &mode, &a, &b, &c, &d) == 5) {
    if (mode == 'w') {
      const mxa::Cd w = mxa::faddeeva_upper({a, b});
      std::printf("%.17g %.17g\n", w.re, w.im);
    } else {
      mxa::Cd e, de;
      mxa::conv_exp(a, b, c, d, &e, &de);
      std::printf("%.17g %.17g %.17g %.17g\n", e.re, e.im, de.re, de.im);
    }
  }
}
'''


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    d = tmp_path_factory.mktemp("resolution")
    src = d / "t.cpp"
    src.write_text(SRC)
    exe = d / "t"
    subprocess.run(["g++", "-O2", "-std=c++17", "-mfma", "-I",
                    os.path.join(ROOT, "paper_1702_06735_amd", "csrc"), "-o", str(exe), str(src)],
                   check=True)
    return str(exe)


def _run(prog, rows):
    inp = "\n".join(" ".join([r[0]] + [repr(float(v)) for v in r[1:]]) for r in rows) + "\n"
    out = subprocess.run([prog], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[float(v) for v in line.split()] for line in out.strip().splitlines()])


def test_faddeeva_against_scipy(prog):
    rng = np.random.default_rng(1)
    z = np.concatenate([rng.uniform(-40, 40, 3000) + 1j * rng.uniform(0, 40, 3000),
                        rng.uniform(-8, 8, 3000) + 1j * rng.uniform(0, 2, 3000),
                        rng.uniform(-3, 3, 2000) + 1j * rng.uniform(0, 1e-3, 2000),
                        np.array([0.0, 1j, 5.0, 1e-8j])])
    out = _run(prog, [("w", v.real, v.imag, 0.0, 0.0) for v in z])
    w = out[:, 0] + 1j * out[:, 1]
    ref = wofz(z)
    assert np.max(np.abs(w - ref) / np.abs(ref)) < 5e-14


def _closed_form(a, t, s):
    """E(a; t) = 1/2 exp(a^2 s^2/2 - a t) erfc(u), u = (a s^2 - t)/(sqrt 2 s),
    with erfc(u) = exp(-u^2) w(i u) for Re u >= 0 and 2 - exp(-u^2) w(-i u)
    otherwise (w from SciPy), so that no factor overflows."""
    u = (a * s * s - t) / (np.sqrt(2.0) * s)
    g = np.exp(-t * t / (2 * s * s))
    if u.real >= 0:
        return 0.5 * g * wofz(1j * u)
    return np.exp(a * a * s * s / 2 - a * t) - 0.5 * g * wofz(-1j * u)


def test_convolved_exponential(prog):
    rng = np.random.default_rng(2)
    G = 1 / 0.4101
    rows, ref, args = [], [], []
    for _ in range(4000):
        s = rng.uniform(0.01, 0.2)
        t = rng.uniform(-5 * s, 8.0)
        x = rng.uniform(-0.5, 0.5) if rng.random() < 0.5 else 0.0
        a = G * (1 + rng.uniform(-0.5, 0.5)) - 1j * G * x
        rows.append(("e", a.real, a.imag, t, s))
        args.append((a, t, s))
    out = _run(prog, rows)
    e = out[:, 0] + 1j * out[:, 1]
    de = out[:, 2] + 1j * out[:, 3]
    ref = np.array([_closed_form(a, t, s) for a, t, s in args])
    scale = np.abs(ref)
    assert np.max(np.abs(e - ref) / scale) < 1e-12
    # dE/da against central differences of the closed form (holomorphic in a)
    h = 1e-5
    fd = np.array([(_closed_form(a + h, t, s) - _closed_form(a - h, t, s)) / (2 * h) for a, t, s in args])
    assert np.max(np.abs(de - fd) / (np.abs(fd) + 1e-3 * scale)) < 1e-6


def test_narrow_resolution_limit(prog):
    # sigma -> 0: E(a; t) -> exp(-a t) for t > 0
    rows = [("e", 2.4, -0.3, t, 1e-6) for t in (0.1, 0.5, 2.0, 5.0)]
    out = _run(prog, rows)
    e = out[:, 0] + 1j * out[:, 1]
    ref = np.exp(-(2.4 - 0.3j) * np.array([0.1, 0.5, 2.0, 5.0]))
    assert np.allclose(e, ref, rtol=1e-9)
