"""Host build of the library's FP64 time functions (csrc/mixfns.h, used on the
device for cosh/sinh of y Gamma t and sin/cos of x Gamma t) checked against
the C math library."""

import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = r'''
#include <cstdio>
#include <cmath>
#include "mixfns.h"
int main() {
  double u;
  while (std::scanf("%lf", &u) == 1) {
    double ch, sh, sn, cs;
    mxa::mix_cosh_sinh(u, &ch, &sh);
    mxa::mix_sincos(u, &sn, &cs);
    std::printf("%.17g %.17g %.17g %.17g\n", ch, sh, sn, cs);
  }
}
'''


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    d = tmp_path_factory.mktemp("mixfns")
    src = d / "t.cpp"
    src.write_text(SRC)
    exe = d / "t"
    subprocess.run(["g++", "-O2", "-std=c++17", "-mfma", "-I",
                    os.path.join(ROOT, "paper_1702_06735_amd", "csrc"), "-o", str(exe), str(src)],
                   check=True)
    return str(exe)


def _run(prog, x):
    out = subprocess.run([prog], input="\n".join(repr(float(v)) for v in x), capture_output=True,
                         text=True, check=True).stdout
    return np.array([[float(t) for t in line.split()] for line in out.splitlines()])


def _ulps(got, ref):
    return np.abs(got - ref) / np.spacing(np.abs(ref))


def test_hyperbolic_against_libm(prog):
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-1, 1, 3000) * 10.0 ** rng.integers(-8, 1, 3000),
                        rng.uniform(-50, 50, 2000), rng.uniform(-700, 700, 500),
                        [0.0, 0.5, -0.5, 0.4999999, 0.5000001]])
    r = _run(prog, x)
    assert np.max(_ulps(r[:, 0], np.cosh(x))) <= 4
    nz = x != 0
    assert np.max(_ulps(r[nz, 1], np.sinh(x[nz]))) <= 4
    assert np.all(r[~nz, 1] == 0)


def test_trigonometric_against_libm(prog):
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-1, 1, 3000) * 10.0 ** rng.integers(-8, 1, 3000),
                        rng.uniform(-50, 50, 2000), rng.uniform(-1e4, 1e4, 500),
                        [0.0, np.pi / 4, np.pi / 2, np.pi, 3 * np.pi / 2, -np.pi / 4]])
    r = _run(prog, x)
    # absolute error against 1: near a zero of sin or cos an ulp count is meaningless
    assert np.max(np.abs(r[:, 2] - np.sin(x))) <= 5e-16
    assert np.max(np.abs(r[:, 3] - np.cos(x))) <= 5e-16
    small = (np.abs(x) < 0.7) & (x != 0)
    assert np.max(_ulps(r[small, 2], np.sin(x[small]))) <= 2
    assert np.max(_ulps(r[small, 3], np.cos(x[small]))) <= 2
