"""The oracle (oracle/oracle.cpp) and the minimiser (csrc/bfgs.h) built on the
host with AddressSanitizer and UndefinedBehaviorSanitizer (g++, CPU only).

The sanitized oracle is linked into a small test program (so that nothing
is preloaded into the Python process): the program reads a model, parameters
and events written by this test, runs the per-event terms, NLL, dual-number
gradient, flavour-tagged NLL and the generator, and writes the results,
which must equal those of the normally built oracle. Any out-of-bounds
access, use after free, signed overflow or other undefined behaviour stops
the program with an error report."""

import os
import struct
import subprocess

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

PROGRAM = r'''
#include "oracle.cpp"
#include <cstdio>
#include <cstdlib>
#include <vector>
template <class T> static void rd(FILE* f, T* p, size_t n) {
  if (n && fread(p, sizeof(T), n, f) != n) { fprintf(stderr, "short input\n"); exit(3); }
}
template <class T> static void wr(FILE* f, const T* p, size_t n) { if (n) fwrite(p, sizeof(T), n, f); }
int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* in = fopen(argv[1], "rb");
  FILE* out = fopen(argv[2], "wb");
  if (!in || !out) return 2;
  int32_t sz, nt, tagged;
  rd(in, &sz, 1);
  if (sz != (int32_t)sizeof(orc_model)) { fprintf(stderr, "model size %d\n", sz); return 4; }
  orc_model m;
  rd(in, &m, 1);
  rd(in, &nt, 1);
  std::vector<double> th(nt);
  rd(in, th.data(), nt);
  int64_t nd, nm;
  rd(in, &nd, 1);
  std::vector<double> pd(nd * 16), td(nd);
  std::vector<int8_t> tag(nd);
  rd(in, pd.data(), nd * 16);
  rd(in, td.data(), nd);
  rd(in, tag.data(), nd);
  rd(in, &nm, 1);
  std::vector<double> pm(nm * 16);
  rd(in, pm.data(), nm * 16);
  double wmax, env;
  rd(in, &wmax, 1);
  rd(in, &env, 1);
  rd(in, &tagged, 1);
  fclose(in);
  std::vector<double> o(4, 0.0), g(nt, 0.0), terms(nd * 5, 0.0);
  int32_t rc[4] = {0, 0, 0, 0};
  if (tagged) {
    rc[0] = orc_nll_tagged(&m, th.data(), nt, pd.data(), td.data(), tag.data(), nd, pm.data(), nm, 1,
                           o.data(), g.data());
    std::vector<double> o2(4);
    rc[1] = orc_nll_tagged(&m, th.data(), nt, pd.data(), td.data(), tag.data(), nd, pm.data(), nm, 1,
                           o2.data(), nullptr);
    o[3] = o2[0];
  } else {
    rc[0] = orc_nll_grad(&m, th.data(), nt, pd.data(), td.data(), nd, pm.data(), nm, 1, o.data(),
                         g.data());
    std::vector<double> o2(4);
    rc[1] = orc_nll(&m, th.data(), nt, pd.data(), td.data(), nd, pm.data(), nm, 1, o2.data());
    o[3] = o2[0];
    rc[2] = orc_event_terms(&m, th.data(), nt, pd.data(), td.data(), nd, 1, terms.data());
  }
  // generator: uniform phase space, and data at theta for models without extensions
  const int64_t nc = 3000;
  std::vector<int64_t> idx(nc), st(3), idx2(nc), st2(3, 0);
  std::vector<double> gp(nc * 16), gp2(nc * 16), gt2(nc);
  rc[3] = orc_generate(&m, th.data(), nt, 1, 77, 5, nc, wmax, 0.0, nc, 1, idx.data(), gp.data(),
                       nullptr, st.data());
  if (env > 0.0)
    rc[3] |= orc_generate(&m, th.data(), nt, 0, 78, 0, nc, wmax, env, nc, 1, idx2.data(), gp2.data(),
                          gt2.data(), st2.data());
  wr(out, rc, 4);
  wr(out, o.data(), 4);
  wr(out, g.data(), nt);
  wr(out, terms.data(), nd * 5);
  wr(out, st.data(), 3);
  wr(out, idx.data(), st[0]);
  wr(out, gp.data(), st[0] * 16);
  wr(out, st2.data(), 3);
  wr(out, gp2.data(), st2[0] * 16);
  wr(out, gt2.data(), st2[0]);
  fclose(out);
  return 0;
}
'''


def _tool(name):
    try:
        subprocess.run([name, "--version"], capture_output=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        pytest.skip(f"{name} not available")


@pytest.fixture(scope="module")
def program(tmp_path_factory):
    _tool("g++")
    d = tmp_path_factory.mktemp("san")
    (d / "drv.cpp").write_text(PROGRAM)
    exe = d / "drv"
    r = subprocess.run(["g++", *SAN, "-std=c++17", "-fopenmp", "-I", os.path.join(ROOT, "oracle"),
                        "-o", str(exe), str(d / "drv.cpp")], capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("no sanitizer runtime: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    return str(exe), d


WMAX = I.genbod_wmax(I.MODEL_FULL["m_D"], (I.MODEL_FULL["m_K"],) + (I.MODEL_FULL["m_pi"],) * 3)


def _case(name):
    """(model, theta, tags or None, data-generation envelope or 0)."""
    base = I.MODEL_SMALL if name in ("small", "resolution") else I.MODEL_FULL
    th = I.make_theta(base, I.draw_coefficients(base, 11))
    if name == "background":
        return I.with_background(base), np.concatenate([th, [0.15]]), None, 0.0
    if name == "cpv":
        return I.with_cp_violation(base), np.concatenate([th, [1.07, 0.2]]), True, 0.0
    if name == "resolution":
        return dict(base, sigma_t=0.06), th, None, 0.0
    return base, th, None, -1.0


@pytest.mark.parametrize("name", ["small", "full", "background", "cpv", "resolution"])
def test_oracle_under_sanitizers(orc, program, name):
    exe, d = program
    model, th, tagged, env = _case(name)
    rng = np.random.default_rng(3)
    nd = 40 if name == "resolution" else 300
    pd = I.phase_space(nd, 31).reshape(nd, 16)
    td = rng.exponential(0.41, nd)
    tags = np.where(rng.random(nd) < 0.5, 1, -1).astype(np.int8)
    pm = I.phase_space(2_000, 32).reshape(-1, 16)
    if env < 0:
        e = orc.event_terms(model, th, I.phase_space(20_000, 33))
        env = 1.2 * float((e[:, 0] + e[:, 1]).max())
    mstruct = orc.OracleModel.from_preset(model)
    blob = (struct.pack("<i", len(bytes(mstruct))) + bytes(mstruct) + struct.pack("<i", th.size)
            + np.asarray(th, "<f8").tobytes() + struct.pack("<q", nd) + pd.astype("<f8").tobytes()
            + td.astype("<f8").tobytes() + tags.tobytes() + struct.pack("<q", len(pm))
            + pm.astype("<f8").tobytes() + struct.pack("<dd", WMAX, env)
            + struct.pack("<i", 1 if tagged else 0))
    (d / f"{name}.in").write_bytes(blob)
    r = subprocess.run([exe, str(d / f"{name}.in"), str(d / f"{name}.out")], capture_output=True,
                       text=True, env=ENV, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    buf = (d / f"{name}.out").read_bytes()
    pos = 0

    def take(dtype, n):
        nonlocal pos
        a = np.frombuffer(buf, dtype=dtype, count=n, offset=pos)
        pos += a.nbytes
        return a

    rc = take("<i4", 4)
    o = take("<f8", 4)
    g = take("<f8", th.size)
    terms = take("<f8", nd * 5).reshape(nd, 5)
    st = take("<i8", 3)
    idx = take("<i8", int(st[0]))
    gp = take("<f8", int(st[0]) * 16)
    st2 = take("<i8", 3)
    gp2 = take("<f8", int(st2[0]) * 16)
    gt2 = take("<f8", int(st2[0]))
    assert not rc.any(), rc
    # the same results as the normally built oracle
    close = lambda a, b: np.allclose(a, b, rtol=1e-12, atol=0.0)
    if tagged:
        v, gr = orc.nll_tagged(model, th, pd, td, tags, pm, grad=True)
        assert close(o[0], v) and close(o[3], v) and close(g, gr)
    else:
        v, gr = orc.nll_grad(model, th, pd, td, pm)
        assert close(o[0], v) and close(o[3], v) and close(g, gr)
        assert close(terms, orc.event_terms(model, th, pd, td))
    ri, rp, _, rst = orc.generate(model, th, "mc", 77, 3000, WMAX, first=5)
    assert tuple(st) == rst and np.array_equal(idx, ri) and np.array_equal(gp, rp.reshape(-1))
    if env > 0:
        _, rp2, rt2, rst2 = orc.generate(model, th, "data", 78, 3000, WMAX, envelope=env)
        assert tuple(st2) == rst2 and np.array_equal(gp2, rp2.reshape(-1))
        assert np.array_equal(gt2, rt2)


def test_minimiser_under_sanitizers(tmp_path):
    """The BFGS state machine with its error phase on the test functions of
    test_bfgs.py, built with the sanitizers."""
    _tool("g++")
    from test_bfgs import SRC
    (tmp_path / "t.cpp").write_text(SRC)
    exe = tmp_path / "t"
    r = subprocess.run(["g++", *SAN, "-std=c++17", "-I",
                        os.path.join(ROOT, "paper_1702_06735_amd", "csrc"), "-o", str(exe),
                        str(tmp_path / "t.cpp")], capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("no sanitizer runtime: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    for args in (["0", "12"], ["1", "10"], ["2", "6"], ["3", "4"], ["4", "12", "1e-4"], ["0", "12", "1e-6"]):
        p = subprocess.run([str(exe), *args], capture_output=True, text=True, env=ENV, timeout=300)
        assert p.returncode == 0 and "runtime error" not in p.stderr, (args, p.stderr[-3000:])
