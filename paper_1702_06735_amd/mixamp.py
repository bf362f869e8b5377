"""ctypes binding of the HIP library ``libmixamp.so`` (declared in
``include/mixamp.h``).

Argument marshalling only: every step of the likelihood runs in the library's
HIP kernels. The library must have been built (``paper_1702_06735_amd.build``);
loading fails loudly otherwise, there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmixamp.so")

MXA_OK = 0
MXA_EINVAL = -1
MXA_ENOMEM = -2
MXA_EDEVICE = -3
MXA_EDOMAIN = -4
MXA_EAGAIN = -5
MXA_ENOTFOUND = -6
MXA_DATA = 0
MXA_MC = 1
MXA_FP64 = 0
MXA_FP32AMP = 1
MXA_DATA_BAR = 2
MXA_MC_DIRECT = 0
MXA_MC_GRAM = 1

PRECISIONS = {"fp64": MXA_FP64, "fp32amp": MXA_FP32AMP, MXA_FP64: MXA_FP64,
              MXA_FP32AMP: MXA_FP32AMP}

#: every symbol include/mixamp.h declares
EXPORTS = (
    "mxa_n_theta", "mxa_create", "mxa_destroy", "mxa_load_events", "mxa_load_events_device",
    "mxa_sample_size", "mxa_set_params", "mxa_nll", "mxa_nll_grad", "mxa_event_terms",
    "mxa_set_stream", "mxa_set_timing", "mxa_kernel_time", "mxa_launch_shape", "mxa_last_error",
    "mxa_set_mc_mode", "mxa_gram",
    "mxa_server_create", "mxa_server_create_streamed", "mxa_fit_submit", "mxa_fit_poll",
    "mxa_fit_wait", "mxa_fit_cancel",
    "mxa_server_stats", "mxa_server_set_graph", "mxa_server_destroy", "mxa_generate", "mxa_nll_multi",
    "mxa_fit", "mxa_nll_grad_noalloc", "mxa_fit_release",
)

MXA_MAX_THETA = 40
FIT_STATUS = {0: "queued", 1: "running", 2: "converged", 3: "max_evals", 4: "failed",
              5: "cancelled"}


class GenStats(C.Structure):
    _fields_ = [("n_candidates", C.c_int64), ("n_phase_space", C.c_int64),
                ("n_exceed", C.c_int64), ("next", C.c_uint64)]

    def to_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class FitRequest(C.Structure):
    _fields_ = [
        ("p4", C.POINTER(C.c_double)), ("t", C.POINTER(C.c_double)), ("n", C.c_int64),
        ("theta0", C.POINTER(C.c_double)), ("scale", C.POINTER(C.c_double)),
        ("max_evals", C.c_int32), ("gtol", C.c_double), ("ftol", C.c_double),
        ("edm_tol", C.c_double), ("errors", C.c_int32), ("gradient", C.c_int32),
        ("events_on_device", C.c_int32),
    ]


class FitResult(C.Structure):
    _fields_ = [
        ("theta", C.c_double * MXA_MAX_THETA), ("nll", C.c_double), ("grad_norm", C.c_double),
        ("n_evals", C.c_int32), ("status", C.c_int32), ("n", C.c_int64),
        ("t_submit_ns", C.c_int64), ("t_start_ns", C.c_int64), ("t_done_ns", C.c_int64),
        ("errors_ok", C.c_int32), ("err", C.c_double * MXA_MAX_THETA),
        ("grad", C.c_double * MXA_MAX_THETA), ("n_points", C.c_int64),
    ]

    def to_dict(self, n_theta):
        return {"theta": np.array(self.theta[:n_theta]), "nll": self.nll,
                "grad_norm": self.grad_norm, "n_evals": self.n_evals,
                "status": FIT_STATUS.get(self.status, str(self.status)), "n": self.n,
                "latency_s": (self.t_done_ns - self.t_submit_ns) * 1e-9,
                "queue_s": (self.t_start_ns - self.t_submit_ns) * 1e-9,
                "t_submit_ns": self.t_submit_ns, "t_start_ns": self.t_start_ns,
                "t_done_ns": self.t_done_ns, "errors_ok": bool(self.errors_ok),
                "err": np.array(self.err[:n_theta]), "grad": np.array(self.grad[:n_theta]),
                "n_points": int(self.n_points)}


class MixampError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mixamp error {code}: {msg}")
        self.code = code


class ModelDesc(C.Structure):
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
    def from_preset(cls, p: dict) -> "ModelDesc":
        m = cls()
        for k in ("m_D", "m_K", "m_pi", "r", "m_ks_ref", "m_rho_ref",
                  "m_k1a", "g_k1a", "m_k1b", "g_k1b"):
            setattr(m, k, float(p[k]))
        m.gamma = 1.0 / float(p["tau"])
        m.n_a, m.n_ab = len(p["comp_a"]), len(p["comp_ab"])
        for i, k in enumerate(p["comp_a"]):
            m.comp_a[i] = int(k)
        for i, k in enumerate(p["comp_ab"]):
            m.comp_ab[i] = int(k)
        m.g_bkg = float(p.get("g_bkg", 0.0))
        m.cpv = 1 if p.get("cpv") else 0
        m.sigma_t = float(p.get("sigma_t", 0.0))
        return m


_lib = None


def load_library(path: str = LIB_PATH):
    """Load ``libmixamp.so`` and declare its prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1702_06735_amd.build.build()")
    # PyTorch ships its own HIP runtime with the same soname. Importing it first
    # makes the dynamic linker bind this library to that copy, so the process
    # holds one HIP runtime (two copies cannot share the GPU).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    i32, i64, vp = C.c_int32, C.c_int64, C.c_void_p
    pd, pi64 = C.POINTER(C.c_double), C.POINTER(C.c_int64)
    pm = C.POINTER(ModelDesc)
    proto = {
        "mxa_n_theta": ([pm], i32),
        "mxa_create": ([pm, i32, vp, C.POINTER(vp)], i32),
        "mxa_destroy": ([vp], i32),
        "mxa_load_events": ([vp, i32, pd, pd, i64], i32),
        "mxa_load_events_device": ([vp, i32, vp, vp, i64], i32),
        "mxa_sample_size": ([vp, i32, pi64], i32),
        "mxa_set_params": ([vp, pd, i32], i32),
        "mxa_nll": ([vp, i32, pd, pd], i32),
        "mxa_nll_grad": ([vp, i32, pd, pd, pd], i32),
        "mxa_nll_grad_noalloc": ([vp, i32, pd, pd, pd], i32),
        "mxa_event_terms": ([vp, i32, i32, pd], i32),
        "mxa_set_stream": ([vp, vp], i32),
        "mxa_set_timing": ([vp, i32], i32),
        "mxa_kernel_time": ([vp, pd, pi64, i32], i32),
        "mxa_launch_shape": ([vp, i32, pi64], i32),
        "mxa_last_error": ([], C.c_char_p),
        "mxa_set_mc_mode": ([vp, i32], i32),
        "mxa_gram": ([vp, i32, pd], i32),
        "mxa_server_create": ([pm, i32, i32, pd, pd, i64, i64, i32, C.POINTER(vp)], i32),
        "mxa_server_create_streamed": ([pm, i32, i32, pd, i64, i64, i32, C.POINTER(vp)], i32),
        "mxa_fit_submit": ([vp, C.POINTER(FitRequest), C.POINTER(C.c_uint64)], i32),
        "mxa_fit_poll": ([vp, C.c_uint64, C.POINTER(FitResult)], i32),
        "mxa_fit_wait": ([vp, C.c_uint64, C.POINTER(FitResult)], i32),
        "mxa_fit_cancel": ([vp, C.c_uint64], i32),
        "mxa_fit_release": ([vp, C.c_uint64], i32),
        "mxa_server_stats": ([vp, pi64], i32),
        "mxa_server_set_graph": ([vp, i32], i32),
        "mxa_server_destroy": ([vp], i32),
        "mxa_nll_multi": ([vp, i32, pd, i32, pd], i32),
        "mxa_fit": ([vp, i32, C.POINTER(FitRequest), C.POINTER(FitResult)], i32),
        "mxa_generate": ([vp, i32, C.c_uint64, C.c_uint64, i64, C.c_double, C.c_double, vp, vp, vp,
                          C.POINTER(GenStats)], i32),
    }
    for name, (args, res) in proto.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != MXA_OK:
        raise MixampError(rc, load_library().mxa_last_error().decode())


def _pd(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _events(p4):
    a = np.ascontiguousarray(p4, dtype=np.float64)
    if a.ndim == 3:
        a = a.reshape(a.shape[0], 16)
    if a.ndim != 2 or a.shape[1] != 16:
        raise ValueError("events must be [n, 4, 4] or [n, 16] float64")
    return a


def _is_cuda_tensor(x) -> bool:
    try:
        import torch
    except ImportError:
        return False
    return isinstance(x, torch.Tensor) and x.device.type == "cuda"


def _check_device_tensor(x, name: str, device: int):
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if x.dtype != torch.float64:
        raise ValueError(f"{name} must be float64, got {x.dtype}")
    if x.device.type != "cuda" or x.device.index != device:
        raise ValueError(f"{name} must be on cuda:{device}, got {x.device}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _current_stream(device: int):
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream(device).cuda_stream
    except ImportError:
        pass
    return None


class Context:
    """One model on one device and stream (``mxa_ctx``)."""

    def __init__(self, model, device: int = 0, stream=None):
        lib = load_library()
        self.model = model if isinstance(model, ModelDesc) else ModelDesc.from_preset(model)
        self.n_theta = lib.mxa_n_theta(C.byref(self.model))
        if self.n_theta < 0:
            _check(self.n_theta)
        if stream is None:
            stream = _current_stream(device)
        h = C.c_void_p()
        _check(lib.mxa_create(C.byref(self.model), device, stream, C.byref(h)))
        self._h = h
        self._lib = lib
        self.device = device
        # output buffers of the evaluation calls and their ctypes pointers, made
        # once (building a ctypes pointer costs microseconds per call); the
        # calls return copies
        self._v = C.c_double()
        self._vp = C.byref(self._v)
        self._g = np.zeros(max(self.n_theta, 1))
        self._gp = _pd(self._g)
        self._d = np.zeros(4)
        self._dp = _pd(self._d)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mxa_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def load_events(self, kind: int, p4, t=None):
        a = _events(p4)
        tt = None if t is None else np.ascontiguousarray(t, dtype=np.float64)
        if tt is not None and tt.shape != (a.shape[0],):
            raise ValueError("t must have one entry per event")
        _check(self._lib.mxa_load_events(self._h, kind, _pd(a), _pd(tt), a.shape[0]))

    def load_events_device(self, kind: int, p4, t=None):
        """``p4``: device tensor [n,4,4] or [n,16] float64, contiguous, on the
        context's device; ``t``: [n] likewise (data kinds). The library reads
        n x 16 and n doubles from the two pointers, so every property is
        checked here before they are handed over."""
        _check_device_tensor(p4, "p4", self.device)
        n = p4.shape[0]
        if tuple(p4.shape[1:]) not in ((4, 4), (16,)):
            raise ValueError(f"p4 must be [n, 4, 4] or [n, 16], got {tuple(p4.shape)}")
        if t is not None:
            _check_device_tensor(t, "t", self.device)
            if tuple(t.shape) != (n,):
                raise ValueError(f"t must be [{n}], got {tuple(t.shape)}")
        _check(self._lib.mxa_load_events_device(self._h, kind, p4.data_ptr() if n else None,
                                                None if t is None or n == 0 else t.data_ptr(), n))

    def sample_size(self, kind: int) -> int:
        n = C.c_int64()
        _check(self._lib.mxa_sample_size(self._h, kind, C.byref(n)))
        return n.value

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        _check(self._lib.mxa_set_params(self._h, _pd(th), th.size))

    def nll(self, precision="fp64", diag=False):
        rc = self._lib.mxa_nll(self._h, PRECISIONS[precision], self._vp, self._dp)
        if rc:
            _check(rc)
        return (self._v.value, self._d.copy()) if diag else self._v.value

    def nll_grad(self, precision="fp64", diag=False):
        rc = self._lib.mxa_nll_grad(self._h, PRECISIONS[precision], self._vp, self._gp, self._dp)
        if rc:
            _check(rc)
        g = self._g[:self.n_theta].copy()
        return (self._v.value, g, self._d.copy()) if diag else (self._v.value, g)

    def nll_grad_noalloc(self, precision="fp64", diag=False):
        """``mxa_nll_grad_noalloc``: as :meth:`nll_grad`, with the reduction
        buffers in the device's fixed scratch array (the call allocates no
        device memory)."""
        rc = self._lib.mxa_nll_grad_noalloc(self._h, PRECISIONS[precision], self._vp, self._gp,
                                            self._dp)
        if rc:
            _check(rc)
        g = self._g[:self.n_theta].copy()
        return (self._v.value, g, self._d.copy()) if diag else (self._v.value, g)

    def fit(self, theta0, scale, precision="fp64", max_evals=150, gtol=1e-3, ftol=0.0,
            edm_tol=0.0, errors=False, central=False):
        """Fit the loaded data sample (``mxa_fit``): parameters with scale > 0
        float; returns the result as a dict (``FitResult.to_dict``)."""
        th = np.ascontiguousarray(theta0, dtype=np.float64)
        sc = np.ascontiguousarray(scale, dtype=np.float64)
        if th.shape != (self.n_theta,) or sc.shape != (self.n_theta,):
            raise ValueError(f"theta0 and scale need {self.n_theta} entries")
        req = FitRequest(None, None, 0, _pd(th), _pd(sc), int(max_evals), float(gtol), float(ftol),
                         float(edm_tol), int(bool(errors)), 1 if central else 0)
        r = FitResult()
        _check(self._lib.mxa_fit(self._h, PRECISIONS[precision], C.byref(req), C.byref(r)))
        return r.to_dict(self.n_theta)

    def nll_multi(self, thetas, precision="fp64"):
        """NLL at each row of ``thetas`` [n_sets, n_theta] (rows share the
        masses and widths): one data pass for all sets, normalisation from the
        MC Gram matrix (``mxa_nll_multi``)."""
        th = np.ascontiguousarray(thetas, dtype=np.float64)
        if th.ndim != 2 or th.shape[1] != self.n_theta:
            raise ValueError(f"thetas must be [n_sets, {self.n_theta}]")
        out = np.zeros(th.shape[0])
        _check(self._lib.mxa_nll_multi(self._h, PRECISIONS[precision], _pd(th), th.shape[0],
                                       _pd(out)))
        return out

    def generate(self, kind: int, n: int, seed: int, first: int = 0, wmax: float = 0.0,
                 envelope: float = 0.0, with_idx: bool = False):
        """First ``n`` kept candidates from ``first`` on (``mxa_generate``):
        uniform phase space (MXA_MC) or pseudo-data at the current parameters
        (MXA_DATA, envelope M_Phi). Returns device tensors (p4 [n,4,4], t [n]
        or None, candidate indices [n] or None) and the statistics."""
        import torch
        dev = torch.device("cuda", self.device)
        p4 = torch.empty((n, 4, 4), dtype=torch.float64, device=dev)
        t = torch.empty(n, dtype=torch.float64, device=dev) if kind == MXA_DATA else None
        idx = torch.empty(n, dtype=torch.int64, device=dev) if with_idx else None
        st = GenStats()
        _check(self._lib.mxa_generate(self._h, kind, int(seed), int(first), int(n), float(wmax),
                                      float(envelope), p4.data_ptr() if n else None,
                                      t.data_ptr() if t is not None and n else None,
                                      idx.data_ptr() if idx is not None and n else None,
                                      C.byref(st)))
        return p4, t, idx, st.to_dict()

    def draw_data(self, theta, n: int, seed: int, n_env: int = 1_000_000, safety: float = 1.2,
                  max_tries: int = 8):
        """Pseudo-data at ``theta`` (Sec. 3.1). The envelope M_Phi is
        ``safety`` times the largest |A|^2 + |Abar|^2 over ``n_env`` uniform
        events (the phase-space stream of the same seed); a draw with any
        candidate above it is repeated with a 1.5x larger one. Leaves
        ``theta`` set. Returns device tensors (p4, t) and the statistics with
        the envelope used."""
        with Context(self.model, self.device) as env:
            env.set_params(theta)
            u, _, _, _ = env.generate(MXA_MC, n_env, seed)
            env.load_events_device(MXA_MC, u)
            terms = env.event_terms(MXA_MC, "fp64")
            del u
        m_phi = safety * float((terms[:, 0] + terms[:, 1]).max())
        self.set_params(theta)
        for _ in range(max_tries):
            p4, t, _, st = self.generate(MXA_DATA, n, seed, envelope=m_phi)
            if st["n_exceed"] == 0:
                st["envelope"] = m_phi
                return p4, t, st
            m_phi *= 1.5
        raise MixampError(MXA_EDOMAIN, "envelope still exceeded after enlarging it")

    def event_terms(self, kind: int, precision="fp64"):
        n = self.sample_size(kind)
        out = np.zeros((n, 5))
        _check(self._lib.mxa_event_terms(self._h, kind, PRECISIONS[precision], _pd(out)))
        return out

    def set_mc_mode(self, mode: int):
        _check(self._lib.mxa_set_mc_mode(self._h, mode))

    def gram(self, precision="fp64"):
        """Complex 8 x 8 Gram matrix sum_j B_k conj(B_l) of the chain amplitudes."""
        out = np.zeros(128)
        _check(self._lib.mxa_gram(self._h, PRECISIONS[precision], _pd(out)))
        return (out[0::2] + 1j * out[1::2]).reshape(8, 8)

    def set_stream(self, stream=None):
        """Issue the following calls on ``stream``: a torch.cuda.Stream, a raw
        hipStream_t handle, or None for torch's current stream of the device."""
        if stream is None:
            stream = _current_stream(self.device)
        elif hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        _check(self._lib.mxa_set_stream(self._h, stream))

    def set_timing(self, on: bool):
        _check(self._lib.mxa_set_timing(self._h, 1 if on else 0))

    def kernel_time(self, reset=True):
        ms, n = C.c_double(), C.c_int64()
        _check(self._lib.mxa_kernel_time(self._h, C.byref(ms), C.byref(n), 1 if reset else 0))
        return ms.value, n.value

    def launch_shape(self, grad=False):
        out = np.zeros(4, dtype=np.int64)
        _check(self._lib.mxa_launch_shape(self._h, 1 if grad else 0,
                                          out.ctypes.data_as(C.POINTER(C.c_int64))))
        return tuple(int(v) for v in out)


def nll_function():
    """``torch.autograd.Function`` over ``Context.nll_grad``: forward returns
    the NLL at theta (float64 CPU tensor), backward returns grad_out * dNLL/dtheta
    from the library's adjoint pass."""
    import torch

    class NLLFunction(torch.autograd.Function):
        @staticmethod
        def forward(fctx, theta, context, precision="fp64"):
            context.set_params(theta.detach().cpu().numpy())
            v, g = context.nll_grad(precision)
            # the gradient goes back on theta's device and dtype
            fctx.save_for_backward(torch.from_numpy(g).to(device=theta.device, dtype=theta.dtype))
            return theta.new_tensor(v)

        @staticmethod
        def backward(fctx, grad_out):
            (g,) = fctx.saved_tensors
            return grad_out * g, None, None

    return NLLFunction


class Server:
    """Fit server (``mxa_server``): continuous batching of NLL fits that share
    one MC normalisation sample. With ``shape`` (the 6 masses and widths) the
    lineshapes are fixed and the MC enters through its Gram matrix
    (``mxa_server_create``); with ``shape=None`` the fits may float them and
    every tick streams the MC sample once for all active fits
    (``mxa_server_create_streamed``)."""

    def __init__(self, model, mc_p4, shape, precision="fp32amp", device=0,
                 hbm_budget=8 << 30, max_slots=64):
        lib = load_library()
        self.model = model if isinstance(model, ModelDesc) else ModelDesc.from_preset(model)
        self.n_theta = lib.mxa_n_theta(C.byref(self.model))
        mc = _events(mc_p4)
        h = C.c_void_p()
        if shape is None:
            _check(lib.mxa_server_create_streamed(C.byref(self.model), device, PRECISIONS[precision],
                                                  _pd(mc), mc.shape[0], int(hbm_budget),
                                                  int(max_slots), C.byref(h)))
        else:
            sh = np.ascontiguousarray(shape, dtype=np.float64)
            assert sh.size == 6
            _check(lib.mxa_server_create(C.byref(self.model), device, PRECISIONS[precision],
                                         _pd(sh), _pd(mc), mc.shape[0], int(hbm_budget),
                                         int(max_slots), C.byref(h)))
        self._h = h
        self._lib = lib
        self._device = device
        self._held = {}  # ticket -> device tensors the server reads in place

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mxa_server_destroy(self._h)
            self._h = None
        self._held = {}

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, p4, t, theta0, scale, max_evals=150, gtol=1e-3, ftol=0.0, edm_tol=0.0,
               errors=False):
        """Queue a fit. ``p4`` ([n, 4, 4] or [n, 16]) and ``t`` ([n]) are host
        arrays, copied here, or float64 CUDA tensors on the server's device,
        which the server reads in place (``events_on_device``): they are kept
        referenced here until the fit's record is released."""
        th = np.ascontiguousarray(theta0, dtype=np.float64)
        sc = np.ascontiguousarray(scale, dtype=np.float64)
        on_device = _is_cuda_tensor(p4) or _is_cuda_tensor(t)
        if on_device:
            import torch
            _check_device_tensor(p4, "p4", self._device)
            _check_device_tensor(t, "t", self._device)
            n = p4.shape[0]
            if not ((p4.dim() == 3 and tuple(p4.shape[1:]) == (4, 4)) or (p4.dim() == 2 and p4.shape[1] == 16)):
                raise ValueError("events must be [n, 4, 4] or [n, 16]")
            if tuple(t.shape) != (n,):
                raise ValueError(f"t must have shape ({n},), got {tuple(t.shape)}")
            torch.cuda.current_stream(self._device).synchronize()  # the events are ready
            ptrs = (C.cast(C.c_void_p(p4.data_ptr()), C.POINTER(C.c_double)),
                    C.cast(C.c_void_p(t.data_ptr()), C.POINTER(C.c_double)))
        else:
            a = _events(p4)
            tt = np.ascontiguousarray(t, dtype=np.float64)
            n = a.shape[0]
            if tt.shape != (n,):
                raise ValueError(f"t must have shape ({n},), got {tt.shape}")
            ptrs = (_pd(a), _pd(tt))
        req = FitRequest(ptrs[0], ptrs[1], n, _pd(th), _pd(sc), int(max_evals), float(gtol), float(ftol),
                         float(edm_tol), int(bool(errors)), 0, int(on_device))
        ticket = C.c_uint64()
        _check(self._lib.mxa_fit_submit(self._h, C.byref(req), C.byref(ticket)))
        if on_device:
            self._held[ticket.value] = (p4, t)
        return ticket.value

    def poll(self, ticket):
        r = FitResult()
        rc = self._lib.mxa_fit_poll(self._h, ticket, C.byref(r))
        if rc == MXA_EAGAIN:
            return None
        _check(rc)
        return r.to_dict(self.n_theta)

    def wait(self, ticket, release=False):
        """Block until the fit has finished; with ``release`` also forget its
        record (``mxa_fit_release``)."""
        r = FitResult()
        _check(self._lib.mxa_fit_wait(self._h, ticket, C.byref(r)))
        if release:
            _check(self._lib.mxa_fit_release(self._h, ticket))
            self._held.pop(ticket, None)
        return r.to_dict(self.n_theta)

    def cancel(self, ticket):
        _check(self._lib.mxa_fit_cancel(self._h, ticket))

    def release(self, ticket):
        """Forget a finished fit's record (``mxa_fit_release``)."""
        _check(self._lib.mxa_fit_release(self._h, ticket))
        self._held.pop(ticket, None)

    def stats(self):
        out = np.zeros(8, dtype=np.int64)
        _check(self._lib.mxa_server_stats(self._h, out.ctypes.data_as(C.POINTER(C.c_int64))))
        return dict(zip(("ticks", "evals", "active", "queued", "hbm_used", "hbm_peak",
                         "active_peak", "records"), (int(v) for v in out)))

    def set_graph(self, on: bool):
        _check(self._lib.mxa_server_set_graph(self._h, 1 if on else 0))
