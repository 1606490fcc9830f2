"""C-ABI contract, checked without a GPU: the library loads, exports every
function include/irgs.h declares, and rejects bad arguments before any
device work (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "irgs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(irgs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2412_15867_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import paper_2412_15867_amd.build as b
        b.build()
    return _lib.lib()


def test_header_lists_the_boundary():
    names = declared_functions()
    for must in ("irgs_scene_create", "irgs_scene_build", "irgs_scene_refit", "irgs_trace",
                 "irgs_trace_backward", "irgs_trace_packed", "irgs_scene_destroy", "irgs_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(L):
    from paper_2412_15867_amd import _lib
    names = declared_functions()
    for n in names:
        assert hasattr(L, n), f"{n} declared in irgs.h but not exported"
        assert n in _lib.SIGNATURES, f"{n} has no binding signature"
    assert set(_lib.SIGNATURES) == set(names)


def test_binding_flags_match_the_header():
    """Every IRGS_FLAG_* of include/irgs.h has the same value in the binding."""
    from paper_2412_15867_amd import _lib
    flags = dict(re.findall(r"#define IRGS_FLAG_([A-Z_]+)\s+(\d+)u", open(HEADER).read()))
    assert len(flags) >= 6
    for name, value in flags.items():
        assert getattr(_lib, "FLAG_" + name) == int(value), name


def test_trace_bytes_count_the_optional_scratch(L):
    """The per-call scratch grows with the ray sort (24 B per ray and more)
    and, for the backward that traces again, with one batch of hit lists."""
    from paper_2412_15867_amd import _lib
    L.irgs_trace_bytes.restype = ctypes.c_size_t
    L.irgs_trace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32]
    R = 1 << 20
    base = L.irgs_trace_bytes(R, 8, 0)
    assert L.irgs_trace_bytes(R, 8, _lib.FLAG_SORT_RAYS) >= base + 24 * R
    assert L.irgs_trace_bytes(R, 8, _lib.FLAG_RECOMPUTE) >= base + R * 256 * 8
    assert L.irgs_trace_bytes(1 << 26, 8, _lib.FLAG_RECOMPUTE) < (5 << 30) + L.irgs_trace_bytes(1 << 26, 8, 0)
    assert L.irgs_trace_bytes(0, 8, _lib.FLAG_SORT_RAYS) == 0


def test_status_strings_and_version(L):
    assert L.irgs_status_str(0) == b"ok"
    assert L.irgs_status_str(-1) == b"invalid argument"
    assert L.irgs_status_str(-4) == b"invalid scene state"
    assert L.irgs_version().startswith(b"irgs-gfx950")


def test_create_rejects_bad_arguments(L):
    from paper_2412_15867_amd import _lib
    h = ctypes.c_void_p()
    s = _lib.Surfels(1, 1, 1, 1, 1)
    assert L.irgs_scene_create(10, 0, ctypes.byref(s), ctypes.byref(h)) == _lib.IRGS_E_INVALID
    assert b"F = 0" in L.irgs_last_error()
    assert L.irgs_scene_create(10, 65, ctypes.byref(s), ctypes.byref(h)) == _lib.IRGS_E_INVALID
    assert L.irgs_scene_create(-1, 3, ctypes.byref(s), ctypes.byref(h)) == _lib.IRGS_E_INVALID
    # leaf references hold a 27-bit position
    assert L.irgs_scene_create((1 << 27) + 1, 3, ctypes.byref(s), ctypes.byref(h)) == _lib.IRGS_E_INVALID
    s0 = _lib.Surfels(None, 1, 1, 1, 1)
    assert L.irgs_scene_create(10, 3, ctypes.byref(s0), ctypes.byref(h)) == _lib.IRGS_E_INVALID
    assert L.irgs_scene_create(10, 3, None, ctypes.byref(h)) == _lib.IRGS_E_INVALID


def test_unbuilt_scene_and_bad_params_are_rejected(L):
    from paper_2412_15867_amd import _lib
    h = ctypes.c_void_p()
    s = _lib.Surfels(1, 1, 1, 1, 1)  # never dereferenced: nothing runs before the checks
    assert L.irgs_scene_create(4, 3, ctypes.byref(s), ctypes.byref(h)) == _lib.IRGS_OK
    p = _lib.Params(16, 3, 1 / 255, 1e-4, 0.0, float("inf"), 3.0, 0, 0)
    out = _lib.Out(1, 1, 1, None, None, None, None, 0)
    assert L.irgs_trace(h, ctypes.byref(p), 4, 1, 1, ctypes.byref(out), None) == _lib.IRGS_E_STATE
    assert b"not built" in L.irgs_last_error()
    p_bad = _lib.Params(3, 3, 1 / 255, 1e-4, 0.0, float("inf"), 3.0, 0, 0)
    assert L.irgs_trace(h, ctypes.byref(p_bad), 4, 1, 1, ctypes.byref(out), None) == _lib.IRGS_E_INVALID
    assert b"k = 3" in L.irgs_last_error()
    p_f = _lib.Params(16, 8, 1 / 255, 1e-4, 0.0, float("inf"), 3.0, 0, 0)
    assert L.irgs_trace(h, ctypes.byref(p_f), 4, 1, 1, ctypes.byref(out), None) == _lib.IRGS_E_INVALID
    assert L.irgs_trace(h, ctypes.byref(p), -1, 1, 1, ctypes.byref(out), None) == _lib.IRGS_E_INVALID
    assert L.irgs_trace(None, ctypes.byref(p), 4, 1, 1, ctypes.byref(out), None) == _lib.IRGS_E_INVALID
    assert L.irgs_scene_refit(h, None) == _lib.IRGS_E_STATE
    assert L.irgs_trace_backward(h, ctypes.byref(p), 4, 1, 1, ctypes.byref(out), None, None, None) in (
        _lib.IRGS_E_STATE, _lib.IRGS_E_INVALID)
    n_int = ctypes.c_int64()
    assert L.irgs_scene_info(h, ctypes.byref(n_int), None) == _lib.IRGS_E_STATE
    assert L.irgs_scene_destroy(h) == _lib.IRGS_OK
    assert L.irgs_scene_destroy(None) == _lib.IRGS_OK


def test_packed_rejects_bad_arguments(L):
    from paper_2412_15867_amd import _lib
    p = _lib.Params(8, 3, 1 / 255, 1e-4, 0.0, float("inf"), 3.0, 0, 0)
    arr = (ctypes.c_void_p * 1)(None)
    assert L.irgs_trace_packed(arr, 1, ctypes.byref(p), None, 0, None) == _lib.IRGS_E_INVALID
    assert L.irgs_trace_packed(None, 0, ctypes.byref(p), None, 0, None) == _lib.IRGS_E_INVALID


def test_sizes_are_reported(L):
    a = L.irgs_scene_bytes(1_000_000, 8)
    assert 100e6 < a < 600e6     # records, binary + wide trees, and the transient build scratch
    assert L.irgs_scene_bytes(0, 8) >= 0
    assert L.irgs_trace_bytes(0, 8, 0) == 0
    assert L.irgs_trace_bytes(4_194_304, 8, 2) > L.irgs_trace_bytes(4_194_304, 8, 0)
