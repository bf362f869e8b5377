"""ctypes shim around the oracle's C++ implementation (``oracle.cpp``).

TEST INFRASTRUCTURE ONLY: see the package docstring. Arrays are float64,
C-contiguous; events are ``[n, 4, 4]`` (K+, pi-(a), pi+, pi-(b); E, px, py, pz)
and decay times ``[n]`` in ps.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liborc.so")

_lib = None


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile ``oracle.cpp`` into ``liborc.so`` with g++ (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OracleModel(C.Structure):
    _fields_ = [
        ("m_D", C.c_double), ("m_K", C.c_double), ("m_pi", C.c_double),
        ("gamma", C.c_double), ("r", C.c_double),
        ("m_ks_ref", C.c_double), ("m_rho_ref", C.c_double),
        ("m_k1a", C.c_double), ("g_k1a", C.c_double),
        ("m_k1b", C.c_double), ("g_k1b", C.c_double),
        ("n_a", C.c_int32), ("n_ab", C.c_int32),
        ("comp_a", C.c_int32 * 8), ("comp_ab", C.c_int32 * 8),
        ("g_bkg", C.c_double), ("cpv", C.c_int32), ("sigma_t", C.c_double),
    ]

    @classmethod
    def from_preset(cls, p: dict) -> "OracleModel":
        m = cls()
        for k in ("m_D", "m_K", "m_pi", "r", "m_ks_ref", "m_rho_ref",
                  "m_k1a", "g_k1a", "m_k1b", "g_k1b"):
            setattr(m, k, float(p[k]))
        m.gamma = 1.0 / float(p["tau"])
        m.n_a = len(p["comp_a"])
        m.n_ab = len(p["comp_ab"])
        for i, k in enumerate(p["comp_a"]):
            m.comp_a[i] = int(k)
        for i, k in enumerate(p["comp_ab"]):
            m.comp_ab[i] = int(k)
        m.g_bkg = float(p.get("g_bkg", 0.0))
        m.cpv = 1 if p.get("cpv") else 0
        m.sigma_t = float(p.get("sigma_t", 0.0))
        return m


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(_LIB)
    d, i32, i64 = C.c_double, C.c_int, C.c_int64
    pd = C.POINTER(C.c_double)
    pm = C.POINTER(OracleModel)
    lib.orc_n_theta.argtypes = [pm]
    lib.orc_q2.argtypes = [d, d, d]
    lib.orc_q2.restype = d
    lib.orc_barrier.argtypes = [i32, d]
    lib.orc_barrier.restype = d
    lib.orc_ls_two_body.argtypes = [d, d, d, d, d, d, pd]
    lib.orc_ls_three_body.argtypes = [i32, d, d, d, d, d, d, d, pd]
    lib.orc_spin_factors.argtypes = [pd, d, d, d, pd]
    lib.orc_basis.argtypes = [pm, pd, i32, pd, pd]
    lib.orc_rate.argtypes = [d] * 8
    lib.orc_rate.restype = d
    lib.orc_rate_integrated.argtypes = [d] * 7
    lib.orc_rate_integrated.restype = d
    lib.orc_event_terms.argtypes = [pm, pd, i32, pd, pd, i64, i32, pd]
    lib.orc_nll.argtypes = [pm, pd, i32, pd, pd, i64, pd, i64, i32, pd]
    lib.orc_nll_grad.argtypes = [pm, pd, i32, pd, pd, i64, pd, i64, i32, pd, pd]
    lib.orc_nll_tagged.argtypes = [pm, pd, i32, pd, pd, C.c_void_p, i64, pd, i64, i32, pd, pd]
    lib.orc_max_threads.argtypes = []
    u32, u64 = C.c_uint32, C.c_uint64
    lib.orc_philox.argtypes = [C.POINTER(u32), u32, u32]
    lib.orc_candidate_uniforms.argtypes = [u64, u64, u32, pd]
    lib.orc_generate.argtypes = [pm, pd, i32, i32, u64, u64, i64, d, d, i64, i32,
                                 C.POINTER(C.c_int64), pd, pd, C.POINTER(C.c_int64)]
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _model(m):
    return m if isinstance(m, OracleModel) else OracleModel.from_preset(m)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} returned {rc}")


def q2(s, ma, mb):
    return load().orc_q2(float(s), float(ma), float(mb))


def barrier(L, z):
    return load().orc_barrier(int(L), float(z))


def ls_two_body(s, m0, g0, ma, mb, r):
    out = np.zeros(2)
    load().orc_ls_two_body(s, m0, g0, ma, mb, r, _p(out))
    return complex(out[0], out[1])


def ls_three_body(L, s, s_r2, mc, m0, g0, m_r2_ref, r):
    out = np.zeros(2)
    load().orc_ls_three_body(L, s, s_r2, mc, m0, g0, m_r2_ref, r, _p(out))
    return complex(out[0], out[1])


def spin_factors(ev, m_D, m_K, m_pi):
    """Raw spin factors of one event per Bose configuration: returns
    (sf[2,7], qD[2,3], s[2,4]) with the D-vertex break-up momenta (VV, a1, K1)
    and the invariant masses squared s(K+ pi_s), s(pi+ pi_o), s(K+ pi_s pi+),
    s(pi- pi+ pi-)."""
    ev = _f64(ev).reshape(16)
    out = np.zeros(28)
    load().orc_spin_factors(_p(ev), m_D, m_K, m_pi, _p(out))
    out = out.reshape(2, 14)
    return out[:, :7].copy(), out[:, 7:10].copy(), out[:, 10:14].copy()


def basis(model, theta, ev):
    """Bose-symmetrised basis amplitudes B_1..B_8 of one event (complex[8])."""
    m = _model(model)
    th = _f64(theta)
    ev = _f64(ev).reshape(16)
    out = np.zeros(16)
    _check(load().orc_basis(C.byref(m), _p(th), th.size, _p(ev), _p(out)), "orc_basis")
    return out[0::2] + 1j * out[1::2]


def rate(A, Ab, x, y, gamma, t):
    return load().orc_rate(A.real, A.imag, Ab.real, Ab.imag, x, y, gamma, t)


def rate_integrated(A, Ab, x, y, gamma):
    return load().orc_rate_integrated(A.real, A.imag, Ab.real, Ab.imag, x, y, gamma)


def event_terms(model, theta, p4, t=None, nthreads=0):
    """Per-event ``[n, 5]``: |A|^2, |Abar|^2, Re(A Abar*), Im(A Abar*), rate.

    The rate is Eq. (1) at ``t`` when times are given, else its integral over t.
    """
    m = _model(model)
    th = _f64(theta)
    p4 = _f64(p4).reshape(-1, 16)
    n = p4.shape[0]
    tt = _f64(t) if t is not None else None
    out = np.zeros((n, 5))
    _check(load().orc_event_terms(C.byref(m), _p(th), th.size, _p(p4), _p(tt), n,
                                  int(nthreads), _p(out)), "orc_event_terms")
    return out


def nll(model, theta, p4_data, t_data, p4_mc, nthreads=0, diag=False):
    """NLL of the data given the model; ``diag`` also returns (Nhat, sum_l, S)."""
    m = _model(model)
    th = _f64(theta)
    pd_ = _f64(p4_data).reshape(-1, 16)
    td = _f64(t_data)
    pm_ = _f64(p4_mc).reshape(-1, 16)
    out = np.zeros(4)
    rc = load().orc_nll(C.byref(m), _p(th), th.size, _p(pd_), _p(td), pd_.shape[0],
                        _p(pm_), pm_.shape[0], int(nthreads), _p(out))
    _check(rc, "orc_nll")
    return (out[0], out[1], out[2], out[3]) if diag else out[0]


def nll_grad(model, theta, p4_data, t_data, p4_mc, nthreads=0):
    """(NLL, dNLL/dtheta) with the gradient from forward-mode dual numbers."""
    m = _model(model)
    th = _f64(theta)
    pd_ = _f64(p4_data).reshape(-1, 16)
    td = _f64(t_data)
    pm_ = _f64(p4_mc).reshape(-1, 16)
    out = np.zeros(4)
    g = np.zeros(th.size)
    rc = load().orc_nll_grad(C.byref(m), _p(th), th.size, _p(pd_), _p(td), pd_.shape[0],
                             _p(pm_), pm_.shape[0], int(nthreads), _p(out), _p(g))
    _check(rc, "orc_nll_grad")
    return out[0], g


def nll_tagged(model, theta, p4_data, t_data, tags, p4_mc, grad=False, nthreads=0, diag=False):
    """NLL (and with ``grad`` the gradient) of flavour-tagged data for a model
    with CP violation in mixing: ``tags`` +1 (D0) or -1 (D0bar event given as
    its CP conjugate)."""
    m = _model(model)
    th = _f64(theta)
    pd_ = _f64(p4_data).reshape(-1, 16)
    td = _f64(t_data)
    tg = np.ascontiguousarray(tags, dtype=np.int8)
    pm_ = _f64(p4_mc).reshape(-1, 16)
    out = np.zeros(4)
    g = np.zeros(th.size) if grad else None
    rc = load().orc_nll_tagged(C.byref(m), _p(th), th.size, _p(pd_), _p(td),
                               tg.ctypes.data_as(C.c_void_p), pd_.shape[0], _p(pm_), pm_.shape[0],
                               int(nthreads), _p(out), _p(g))
    _check(rc, "orc_nll_tagged")
    if grad:
        return out[0], g
    return (out[0], out[1], out[2], out[3]) if diag else out[0]


def max_threads():
    return load().orc_max_threads()


def philox(ctr, key):
    """One Philox4x32-10 block of the 4-word counter ``ctr`` under the 2-word
    ``key``; returns the 4 output words."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    load().orc_philox(c, int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF)
    return [int(v) for v in c]


def candidate_uniforms(seed, i, stream):
    """The twelve uniforms of candidate ``i`` of a sample."""
    u = np.zeros(12)
    load().orc_candidate_uniforms(int(seed), int(i), int(stream), _p(u))
    return u


def generate(model, theta, kind, seed, n_cand, wmax, envelope=0.0, first=0, max_out=None,
             nthreads=0):
    """Candidates ``first .. first+n_cand-1`` of a pseudo-experiment.

    ``kind`` "mc" (uniform phase space) or "data" (Eq. (1) at ``theta`` with
    the envelope ``M_Phi = envelope``). Returns (idx, p4 [k,4,4], t or None,
    stats) for the kept candidates in order (at most ``max_out``), with stats =
    (kept, kept by GENBOD, envelope exceedances)."""
    m = _model(model)
    data = kind == "data"
    th = _f64(theta) if data else np.zeros(1)
    n_cand = int(n_cand)
    cap = n_cand if max_out is None else int(max_out)
    idx = np.zeros(max(cap, 1), dtype=np.int64)
    p4 = np.zeros((max(cap, 1), 16))
    t = np.zeros(max(cap, 1)) if data else None
    st = np.zeros(3, dtype=np.int64)
    rc = load().orc_generate(C.byref(m), _p(th), th.size, 0 if data else 1, int(seed), int(first),
                             n_cand, float(wmax), float(envelope), cap, int(nthreads),
                             idx.ctypes.data_as(C.POINTER(C.c_int64)), _p(p4), _p(t),
                             st.ctypes.data_as(C.POINTER(C.c_int64)))
    _check(rc, "orc_generate")
    k = int(min(st[0], cap))
    return (idx[:k], p4[:k].reshape(k, 4, 4), t[:k] if data else None,
            tuple(int(v) for v in st))
