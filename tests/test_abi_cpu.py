"""The C-ABI library loads and exports every entry point its header declares;
host-side argument checks answer without touching the device.  CPU only:
nothing here launches a kernel."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phasemask.h")
LIB = os.path.join(ROOT, "paper_1302_0120_amd", "libphasemask.so")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(phasemask_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libphasemask.so is not built (run python -m paper_1302_0120_amd.build)")
    import torch  # noqa: F401  (same HIP runtime as the product binding)
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for must in ("phasemask_create", "phasemask_solve", "phasemask_error", "phasemask_destroy"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    from paper_1302_0120_amd import binding
    assert sorted(binding._SIGNATURES) == _declared_functions()


def test_status_strings(lib):
    lib.phasemask_status_string.restype = ctypes.c_char_p
    for code, tag in [(0, b"PM_OK"), (-1, b"PM_EINVAL"), (-2, b"PM_EUNSUPPORTED"),
                      (-3, b"PM_ENOMEM"), (-4, b"PM_EDEVICE"), (-5, b"PM_ESTATE")]:
        assert lib.phasemask_status_string(code).startswith(tag)


def test_host_side_argument_errors(lib):
    """Rejected before any HIP call: NULL out, bad sizes, NULL handles."""
    lib.phasemask_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                     ctypes.c_uint, ctypes.c_void_p]
    lib.phasemask_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p(1234)
    assert lib.phasemask_create(None, 64, 64, 0, None) == -1
    for hh, ww in [(48, 64), (64, 8), (8192, 64), (64, 0), (-64, 64), (64, 4097), (700, 800),
                   (600, 1000), (720, 1280), (1080, 1000)]:
        assert lib.phasemask_create(ctypes.byref(h), hh, ww, 0, None) == -2
        assert h.value is None
        msg = lib.phasemask_last_error()
        assert b"power" in msg and b"600" in msg and b"800" in msg and b"1920" in msg
    assert lib.phasemask_create(ctypes.byref(h), 64, 64, 0x80, None) == -1
    assert lib.phasemask_destroy(None) == -1
    lib.phasemask_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_void_p]
    assert lib.phasemask_solve(None, None, None, 1, None, None) == -1
    assert lib.phasemask_error(None, None, None, None) == -1
    assert lib.phasemask_fft2(None, None, None, 0) == -1
    assert lib.phasemask_set_stream(None, None) == -1
    lib.phasemask_set_illumination.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.phasemask_set_illumination(None, None) == -1
    lib.phasemask_workspace_bytes.restype = ctypes.c_size_t
    assert lib.phasemask_workspace_bytes(None) == 0


def test_batched_host_side_argument_errors(lib):
    lib.phasemask_create_batched.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                             ctypes.c_uint, ctypes.c_void_p]
    h = ctypes.c_void_p(99)
    hs = (ctypes.c_int * 2)(256, 512)
    ws = (ctypes.c_int * 2)(256, 2048)
    assert lib.phasemask_create_batched(None, 2, hs, hs, 0, None) == -1
    assert lib.phasemask_create_batched(ctypes.byref(h), 0, hs, hs, 0, None) == -1
    assert lib.phasemask_create_batched(ctypes.byref(h), 2, hs, ws, 0, None) == -2
    assert h.value is None
    small = (ctypes.c_int * 1)(32)
    assert lib.phasemask_create_batched(ctypes.byref(h), 1, small, small, 0, None) == -2
    lib.phasemask_solve_batched.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_void_p, ctypes.c_void_p]
    assert lib.phasemask_solve_batched(None, None, None, 1, None, None) == -1


def test_handles_that_are_not_live_plans(lib):
    """A pointer that is not a live plan (never created, or destroyed) is
    refused with PM_ESTATE before it is dereferenced; the size queries answer
    0 / -1.  (The GPU tests destroy real plans and call them again.)"""
    bogus = ctypes.c_void_p(0x12345678)
    f = ctypes.c_void_p(0x1000)
    lib.phasemask_solve.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int] + [ctypes.c_void_p] * 2
    assert lib.phasemask_solve(bogus, f, f, 3, f, None) == -5
    lib.phasemask_destroy.argtypes = [ctypes.c_void_p]
    assert lib.phasemask_destroy(bogus) == -5
    lib.phasemask_set_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.phasemask_set_stream(bogus, None) == -5
    lib.phasemask_batch_config.argtypes = [ctypes.c_void_p] * 4
    assert lib.phasemask_batch_config(bogus, None, None, None) == -5
    lib.phasemask_workspace_bytes.argtypes = [ctypes.c_void_p]
    lib.phasemask_workspace_bytes.restype = ctypes.c_size_t
    assert lib.phasemask_workspace_bytes(bogus) == 0
    lib.phasemask_batch_schedule.argtypes = [ctypes.c_void_p]
    assert lib.phasemask_batch_schedule(bogus) == -1
    lib.phasemask_last_error.restype = ctypes.c_char_p
    assert b"not a live plan" in lib.phasemask_last_error()
