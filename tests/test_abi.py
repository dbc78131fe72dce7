"""Host-only checks of the C ABI: the library loads, exports every declared
entry point, and rejects invalid input before touching a device."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2601_02172_amd as pkg
from paper_2601_02172_amd import xfft as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "xfft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xfft_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    lib = X._lib()
    names = _declared()
    assert "xfft_setup" in names and "xfft_solve" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == sorted(X.EXPORTS)


def test_default_options_and_strerror():
    o = pkg.default_options()
    assert o.rtol == 1e-10 and o.precision == X.XFFT_FP64 and o.snap_eps == 1e-6 and o.batch == 1
    lib = X._lib()
    for code in (0, 1, -1, -2, -3, -4):
        assert len(lib.xfft_strerror(code)) > 0


def _setup_rc(n, length, L, ph, lame, opt=None):
    lib = X._lib()
    n = np.ascontiguousarray(n, dtype=np.int32)
    length = np.ascontiguousarray(length, dtype=np.float64)
    L = np.ascontiguousarray(L, dtype=np.float64)
    ph = np.ascontiguousarray(ph, dtype=np.int32)
    lame = np.ascontiguousarray(lame, dtype=np.float64)
    h = ctypes.c_void_p()
    rc = lib.xfft_setup(X._ip(n), X._dp(length), X._dp(L), X._ip(ph), lame.shape[0], X._dp(lame),
                        None if opt is None else ctypes.byref(opt), ctypes.byref(h))
    if rc == 0:
        lib.xfft_destroy(h)
    return rc


@pytest.mark.parametrize("case", ["odd", "prime", "small", "noncubic", "nan", "phase", "mu", "bulk", "huge",
                                  "fft_z", "fft_x", "fft_y"])
def test_setup_rejects_invalid_input(case):
    n = [8, 8, 8]
    length = [8.0, 8.0, 8.0]
    N = 512
    L = np.ones(N)
    ph = np.zeros(N, dtype=np.int32)
    lame = np.array([[1.0, 0.5]])
    if case == "odd":
        n = [9, 8, 8]
        L = np.ones(576); ph = np.zeros(576, dtype=np.int32)
    elif case == "prime":
        n = [10, 8, 8]
        L = np.ones(640); ph = np.zeros(640, dtype=np.int32)
    elif case == "small":
        n = [2, 8, 8]
        L = np.ones(128); ph = np.zeros(128, dtype=np.int32)
    elif case == "noncubic":
        length = [8.0, 8.0, 9.0]
    elif case == "nan":
        L[17] = np.nan
    elif case == "phase":
        ph[3] = 1
    elif case == "mu":
        lame = np.array([[1.0, 0.0]])
    elif case == "bulk":
        lame = np.array([[-1.0, 0.5]])
    elif case in ("fft_z", "fft_x", "fft_y"):
        # line FFTs beyond one workgroup of the generic passes: 3 x 1536 / 2
        # butterflies along z, 2592 / 2 along x or y
        n = {"fft_z": [16, 16, 1536], "fft_x": [2592, 16, 16], "fft_y": [16, 2592, 16]}[case]
        length = [float(v) for v in n]
        L = np.ones(int(np.prod(n))); ph = np.zeros(int(np.prod(n)), dtype=np.int32)
    elif case == "huge":
        # 3 N doubles of one load above 4 GiB: rejected before the level set is read
        n = [1024, 1024, 1024]
        length = [1024.0] * 3
    assert _setup_rc(n, length, L, ph, lame) == X.XFFT_EINVAL


@pytest.mark.parametrize("scheme,precision", [(4, X.XFFT_FP64), (-1, X.XFFT_FP64), (1, X.XFFT_MIXED),
                                              (2, X.XFFT_MIXED), (3, X.XFFT_MIXED)])
def test_setup_rejects_invalid_scheme(scheme, precision):
    # options are checked before any device call; only linear CG runs inside the mixed refinement
    o = pkg.default_options()
    assert o.scheme == 0
    o.scheme, o.precision = scheme, precision
    assert _setup_rc([8, 8, 8], [8.0] * 3, np.ones(512), np.zeros(512, dtype=np.int32), np.array([[1.0, 0.5]]),
                     o) == X.XFFT_EINVAL


@pytest.mark.parametrize("disc", [2, -1])
def test_setup_rejects_invalid_discretization(disc):
    o = pkg.default_options()
    assert o.discretization == 0
    o.discretization = disc
    assert _setup_rc([8, 8, 8], [8.0] * 3, np.ones(512), np.zeros(512, dtype=np.int32), np.array([[1.0, 0.5]]),
                     o) == X.XFFT_EINVAL


def test_setup_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc = _setup_rc([8, 8, 8], [8.0] * 3, np.ones(512), np.zeros(512, dtype=np.int32), np.array([[1.0, 0.5]]))
    assert rc == X.XFFT_EDEVICE
