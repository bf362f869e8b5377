"""Host-side checks of the C-ABI library (no GPU compute): it loads, exports
every symbol the header declares, and rejects bad arguments with status codes."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1702_06735_amd import inputs as I
from paper_1702_06735_amd import mixamp as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mixamp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mxa_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(M.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = M.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_n_theta_and_model_validation():
    lib = M.load_library()
    assert lib.mxa_n_theta(C.byref(M.ModelDesc.from_preset(I.MODEL_FULL))) == 36
    assert lib.mxa_n_theta(C.byref(M.ModelDesc.from_preset(I.MODEL_SMALL))) == 16
    bad = M.ModelDesc.from_preset(I.MODEL_FULL)
    bad.comp_a[1] = bad.comp_a[0]  # duplicate chain
    assert lib.mxa_n_theta(C.byref(bad)) == M.MXA_EINVAL
    assert b"distinct" in lib.mxa_last_error()
    bad = M.ModelDesc.from_preset(I.MODEL_FULL)
    bad.comp_ab[0] = 9
    assert lib.mxa_n_theta(C.byref(bad)) == M.MXA_EINVAL


def test_null_arguments_are_rejected():
    lib = M.load_library()
    assert lib.mxa_create(None, 0, None, None) == M.MXA_EINVAL
    assert lib.mxa_nll(None, 0, None, None) == M.MXA_EINVAL
    assert lib.mxa_set_params(None, None, 0) == M.MXA_EINVAL
    assert lib.mxa_set_stream(None, None) == M.MXA_EINVAL
    assert lib.mxa_destroy(None) == M.MXA_OK


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(M.MixampError) as e:
        M.Context(I.MODEL_FULL, device=0, stream=None)
    assert e.value.code == M.MXA_EDEVICE


def test_streamed_server_rejects_bad_arguments_before_the_device():
    lib = M.load_library()
    model = M.ModelDesc.from_preset(I.MODEL_FULL)
    h = C.c_void_p()
    assert lib.mxa_server_create_streamed(C.byref(model), 0, M.PRECISIONS["fp64"], None, 10,
                                          1 << 20, 4, C.byref(h)) == M.MXA_EINVAL
    assert b"MC sample" in lib.mxa_last_error()
    mc = np.zeros((4, 16))
    assert lib.mxa_server_create_streamed(C.byref(model), 0, 7, mc.ctypes.data_as(
        C.POINTER(C.c_double)), 4, 1 << 20, 4, C.byref(h)) == M.MXA_EINVAL
    assert lib.mxa_server_create_streamed(C.byref(model), 0, M.PRECISIONS["fp64"], mc.ctypes.data_as(
        C.POINTER(C.c_double)), 4, 1 << 20, 0, C.byref(h)) == M.MXA_EINVAL
    # the fixed-lineshape server still needs its shape
    assert lib.mxa_server_create(C.byref(model), 0, M.PRECISIONS["fp64"], None, mc.ctypes.data_as(
        C.POINTER(C.c_double)), 4, 1 << 20, 4, C.byref(h)) == M.MXA_EINVAL
    assert b"shape" in lib.mxa_last_error()


def test_device_tensor_checks_reject_before_any_library_call():
    # the binding hands raw device pointers to the library, which reads n x 16
    # doubles: a wrong dtype, device or layout must be refused in Python
    import torch
    with pytest.raises(ValueError, match="float64"):
        M._check_device_tensor(torch.zeros(4, 16, dtype=torch.float32), "p4", 0)
    with pytest.raises(ValueError, match="cuda:0"):
        M._check_device_tensor(torch.zeros(4, 16, dtype=torch.float64), "p4", 0)
    with pytest.raises(TypeError):
        M._check_device_tensor(np.zeros((4, 16)), "p4", 0)
