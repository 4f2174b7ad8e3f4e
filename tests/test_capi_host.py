"""Host-only checks of the C ABI: the library loads, exports every function that
include/gsht.h declares, and rejects invalid arguments before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsht.h")
LIB = os.path.join(ROOT, "paper_2304_10431_amd", "libgsht.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char|const char)\s*\*?\s*(gsht_\w+)\s*\(", src, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libgsht.so is not built (run `python -m paper_2304_10431_amd.build`)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gsht_synth_general", "gsht_adjoint_synth_general", "gsht_last_error",
                     "gsht_plan_create", "gsht_plan_synth", "gsht_plan_adjoint",
                     "gsht_plan_destroy", "gsht_legendre_rings", "gsht_legendre_rings_adjoint"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _create(lib, lmax, mmax, spin, npts, eps, prec, theta=None, phi=None):
    lib.gsht_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
    h = ctypes.c_void_p(0)
    rc = lib.gsht_plan_create(ctypes.byref(h), lmax, mmax, spin, theta, phi, npts, eps, prec, None)
    return rc, h


@pytest.mark.parametrize("args,code", [
    ((-1, 0, 0, 10, 1e-10, 0), -1),          # lmax < 0
    ((10, 11, 0, 10, 1e-10, 0), -1),         # mmax > lmax
    ((10, -1, 0, 10, 1e-10, 0), -1),         # mmax < 0
    ((10, 10, 11, 10, 1e-10, 0), -1),        # spin > lmax
    ((10, 10, -2, 10, 1e-10, 0), -1),        # spin < 0
    ((10, 10, 0, -5, 1e-10, 0), -1),         # npts < 0
    ((10, 10, 0, 10, 1e-14, 0), -1),         # epsilon below the FP64 range
    ((10, 10, 0, 10, 1e-6, 1), -1),          # epsilon below the FP32 range
    ((10, 10, 0, 10, 0.5, 0), -1),           # epsilon above 0.1
    ((10, 10, 0, 10, float("nan"), 0), -1),  # NaN epsilon
    ((10, 10, 0, 10, 1e-10, 7), -1),         # unknown precision
    ((10, 10, 0, 1 << 31, 1e-10, 0), -4),    # npts beyond the int32 point index
    ((10, 10, 0, 10, 1e-10, 0), -1),         # NULL theta/phi with npts > 0
])
def test_invalid_arguments_rejected_on_host(lib, args, code):
    lib.gsht_last_error.restype = ctypes.c_char_p
    rc, h = _create(lib, *args)
    assert rc == code
    assert h.value is None
    assert lib.gsht_last_error().decode() != ""


def test_null_plan_rejected(lib):
    lib.gsht_plan_synth.argtypes = [ctypes.c_void_p] * 4
    assert lib.gsht_plan_synth(None, None, None, None) == -1
    lib.gsht_plan_destroy.argtypes = [ctypes.c_void_p]
    lib.gsht_plan_destroy(None)  # ignored


def test_stage_names(lib):
    lib.gsht_stage_name.restype = ctypes.c_char_p
    n = lib.gsht_num_stages()
    names = [lib.gsht_stage_name(i).decode() for i in range(n)]
    assert "legendre_synth" in names and "legendre_adj" in names and "spread" in names
    assert lib.gsht_stage_name(n).decode() == ""


def test_sigma_and_point_moving_entries_reject_on_host(lib):
    """The oversampling entries check sigma and the arguments before any device work;
    moving points checks the plan pointer and the capacity."""
    lib.gsht_last_error.restype = ctypes.c_char_p
    P = ctypes.POINTER(ctypes.c_void_p)
    lib.gsht_plan_create_sigma.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_void_p]
    lib.gsht_plan_create_tuned.argtypes = lib.gsht_plan_create_sigma.argtypes[:9] + [ctypes.c_void_p]
    h = ctypes.c_void_p(0)
    for sigma in (1.7, 1.0, 3.0, float("nan")):
        assert lib.gsht_plan_create_sigma(ctypes.byref(h), 10, 10, 0, None, None, 10, 1e-10, 0,
                                          sigma, None) == -1
        assert "sigma must be" in lib.gsht_last_error().decode()
        assert h.value is None
    # valid sigma, invalid arguments: the same checks as gsht_plan_create
    assert lib.gsht_plan_create_sigma(ctypes.byref(h), 10, 11, 0, None, None, 10, 1e-10, 0,
                                      1.5, None) == -1
    assert lib.gsht_plan_create_tuned(ctypes.byref(h), 10, 10, 0, None, None, 10, 1e-14, 0,
                                      None) == -1
    assert lib.gsht_plan_create_tuned(None, 10, 10, 0, None, None, 10, 1e-10, 0, None) == -1
    assert h.value is None
    lib.gsht_plan_set_points.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_void_p]
    assert lib.gsht_plan_set_points(None, None, None, 0, None) == -1


def test_noalloc_refuses_sizes_beyond_its_scratch(lib):
    """The allocation-free entry point refuses, before any device work, a size whose
    tables exceed its fixed scratch (lmax 4096, spin 2 needs about 470 MB)."""
    f = lib.gsht_legendre_rings_adjoint_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                  ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.gsht_last_error.restype = ctypes.c_char_p
    rc = f(ctypes.c_void_p(16), 4096, 4096, 2, 4117, 0, ctypes.c_void_p(16), None)
    assert rc == -1
    assert b"scratch" in lib.gsht_last_error()
    rc = f(None, 64, 64, 2, 70, 0, ctypes.c_void_p(16), None)   # NULL input
    assert rc == -1
