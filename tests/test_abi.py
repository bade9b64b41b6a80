"""C-ABI checks that need no GPU: the library loads, exports every function
the public headers declare, and rejects bad arguments before any device
call (so these run on a CPU-only host)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the library under test: the regular build, or (set by the sanitizer test)
# the host-sanitized one
LIB = os.environ.get("WSFFT_ABI_LIB") or os.path.join(ROOT, "paper_2209_15040_amd", "libwsfft.so")

OK, INVALID, UNSUPPORTED, NULLPTR, MISALIGNED, OOM, NODEV, HIPERR, BADPLAN, WRONGDEV = range(10)


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(wsfft_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2209_15040_amd import build
        build.build(incremental=True)
    L = ctypes.CDLL(LIB)
    L.wsfft_plan_create.restype = ctypes.c_void_p
    L.wsfft_plan_create.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_int, ctypes.c_int]
    L.wsfft_plan_create_ex.restype = ctypes.c_void_p
    L.wsfft_plan_create_ex.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_int, ctypes.c_int, ctypes.c_uint]
    L.wsfft_status_string.restype = ctypes.c_char_p
    for f in ("wsfft_execute", "wsfft_execute_adjoint", "wsfft_execute_inverse"):
        getattr(L, f).argtypes = [ctypes.c_void_p] * 4
    L.wsfft_plan_work_bytes.restype = ctypes.c_int64
    L.wsfft_plan_work_bytes.argtypes = [ctypes.c_void_p]
    for f in ("wsfft_plan_scale_log2", "wsfft_plan_num_passes"):
        getattr(L, f).argtypes = [ctypes.c_void_p]
    L.wsfft_plan_describe.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t]
    L.wsfft_plan_destroy.argtypes = [ctypes.c_void_p]
    L.wsfft_real_to_complex.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    L.wsfft_complex_real_part.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    L.wsfft_poisson_symbol.argtypes = [ctypes.c_void_p] + [ctypes.c_int64] * 3 + [ctypes.c_void_p]
    return L


def test_headers_declare_the_named_entry_points():
    names = declared_functions()
    for must in ("wsfft_plan_create", "wsfft_execute", "wsfft_execute_adjoint",
                 "wsfft_execute_batched", "wsfft_plan_destroy", "wsfft_get_last_error"):
        assert must in names


def test_library_exports_every_declared_function(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("dims,dtype,sign,want", [
    ((0, 1, 1), 0, -1, INVALID),
    ((8, -2, 1), 0, -1, INVALID),
    ((8, 8, 8), 0, 0, INVALID),
    ((8, 8, 8), 0, 2, INVALID),
    ((8, 8, 8), 3, -1, INVALID),
    ((8, 8, 8), -1, -1, INVALID),
    ((5, 8, 8), 0, -1, UNSUPPORTED),
    ((8, 7, 8), 1, -1, UNSUPPORTED),
    ((8, 8, 96 * 7), 2, 1, UNSUPPORTED),
    ((2 ** 21, 1, 1), 0, -1, UNSUPPORTED),
    ((1 << 14, 1 << 14, 1 << 14), 0, -1, UNSUPPORTED),   # 2^42 elements
])
def test_plan_create_rejects(lib, dims, dtype, sign, want):
    assert lib.wsfft_plan_create(*dims, dtype, sign) is None
    assert lib.wsfft_get_last_error() == want


def test_unknown_flag_rejected(lib):
    assert lib.wsfft_plan_create_ex(8, 8, 8, 0, -1, 0x80) is None
    assert lib.wsfft_get_last_error() == INVALID


@pytest.mark.parametrize("dtype", [0, 2])
def test_fp16_math_flag_only_for_fp16_storage(lib, dtype):
    assert lib.wsfft_plan_create_ex(8, 8, 8, dtype, -1, 4) is None   # WSFFT_FLAG_FP16_MATH
    assert lib.wsfft_get_last_error() == INVALID


def test_valid_plan_without_device_reports_no_device(lib):
    if os.environ.get("WSFFT_ABI_NO_TORCH"):
        if os.environ.get("HIP_VISIBLE_DEVICES") != "":
            pytest.skip("device visibility unknown without torch")
    else:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a device is visible")
    assert lib.wsfft_plan_create(512, 512, 512, 0, -1) is None
    assert lib.wsfft_get_last_error() == NODEV


def test_execute_rejects_invalid_plans(lib):
    bogus = ctypes.c_void_p(0x1000)
    for f in ("wsfft_execute", "wsfft_execute_adjoint", "wsfft_execute_inverse"):
        assert getattr(lib, f)(None, 0x1000, 0x2000, None) == BADPLAN
        assert getattr(lib, f)(bogus, 0x1000, 0x2000, None) == BADPLAN
    assert lib.wsfft_plan_scale_log2(None) == -1
    assert lib.wsfft_plan_num_passes(bogus) == -1
    assert lib.wsfft_plan_work_bytes(bogus) == -1
    buf = ctypes.create_string_buffer(64)
    assert lib.wsfft_plan_describe(bogus, buf, 64) == BADPLAN
    lib.wsfft_plan_destroy(None)     # ignored
    lib.wsfft_plan_destroy(bogus)    # unknown handle: ignored, no crash


def test_execute_batched_argument_checks(lib):
    f = lib.wsfft_execute_batched
    f.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    assert f(-1, None, None, None, 0, None) == INVALID
    assert f(0, None, None, None, 0, None) == OK
    assert f(2, None, None, None, 0, None) == NULLPTR
    arr = (ctypes.c_void_p * 1)(0x1000)
    plans = (ctypes.c_void_p * 1)(None)
    assert f(1, plans, arr, arr, 0, None) == BADPLAN


def test_tune_batched_argument_checks(lib):
    f = lib.wsfft_tune_batched
    f.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    assert f(-1, None, None, None, 0, None) == INVALID
    assert f(2, None, None, None, 0, None) == NULLPTR
    arr = (ctypes.c_void_p * 1)(0x1000)
    plans = (ctypes.c_void_p * 1)(None)
    assert f(1, plans, arr, arr, 0, None) == BADPLAN


def test_pointwise_argument_checks(lib):
    assert lib.wsfft_real_to_complex(0x1000, 0x2000, -1, None) == INVALID
    assert lib.wsfft_real_to_complex(None, 0x2000, 0, None) == OK
    assert lib.wsfft_real_to_complex(None, 0x2000, 5, None) == NULLPTR
    assert lib.wsfft_real_to_complex(0x1002, 0x2000, 5, None) == MISALIGNED
    assert lib.wsfft_real_to_complex(0x1000, 0x2004, 5, None) == MISALIGNED
    assert lib.wsfft_complex_real_part(0x1004, 0x2000, 5, None) == MISALIGNED
    assert lib.wsfft_poisson_symbol(0x1000, 0, 4, 4, None) == INVALID
    assert lib.wsfft_poisson_symbol(None, 4, 4, 4, None) == NULLPTR
    assert lib.wsfft_poisson_symbol(0x1004, 4, 4, 4, None) == MISALIGNED


def test_poisson_solve_argument_checks(lib):
    f = lib.wsfft_poisson_solve
    f.argtypes = [ctypes.c_void_p] * 5
    bogus = ctypes.c_void_p(0x1000)
    assert f(None, 0x1000, 0x2000, 0x3000, None) == BADPLAN
    assert f(bogus, 0x1000, 0x2000, 0x3000, None) == BADPLAN


def test_status_strings(lib):
    for s in range(10):
        assert lib.wsfft_status_string(s)
    assert lib.wsfft_status_string(OK) == b"success"
    assert lib.wsfft_status_string(99) == b"unknown status"


@pytest.mark.parametrize("dims,flags,want", [
    ((0, 4, 4), 0, INVALID),
    ((8, 8, 8), 1, INVALID),            # no flags are defined for real plans
    ((9, 8, 8), 0, UNSUPPORTED),        # odd real axis
    ((2, 8, 8), 0, UNSUPPORTED),        # nx < 4
    ((65536, 1, 1), 0, UNSUPPORTED),    # nx/2 longer than one contiguous pass
    ((10, 8, 8), 0, UNSUPPORTED),       # factor 5
    ((8, 8, 7), 0, UNSUPPORTED),
])
def test_plan_create_real_rejects(lib, dims, flags, want):
    f = lib.wsfft_plan_create_real
    f.restype = ctypes.c_void_p
    f.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_uint]
    assert f(*dims, flags) is None
    assert lib.wsfft_get_last_error() == want


@pytest.mark.parametrize("dims,pitch,want", [
    ((8, 8, 8), 4, INVALID),            # pitch below nx/2 + 1
    ((8, 8, 8), -1, INVALID),
    ((8, 8, 8), 2 ** 21, INVALID),
    ((9, 8, 8), 16, UNSUPPORTED),       # odd real axis
])
def test_plan_create_real_ex_rejects(lib, dims, pitch, want):
    f = lib.wsfft_plan_create_real_ex
    f.restype = ctypes.c_void_p
    f.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_uint, ctypes.c_int64]
    assert f(*dims, 0, pitch) is None
    assert lib.wsfft_get_last_error() == want


def test_real_calls_reject_invalid_plans(lib):
    bogus = ctypes.c_void_p(0x1000)
    for name in ("wsfft_execute_r2c", "wsfft_execute_c2r", "wsfft_execute_c2r_inverse"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_void_p] * 4
        assert f(None, 0x1000, 0x2000, None) == BADPLAN
        assert f(bogus, 0x1000, 0x2000, None) == BADPLAN
    lib.wsfft_plan_is_real.argtypes = [ctypes.c_void_p]
    assert lib.wsfft_plan_is_real(bogus) == -1


def test_batch_spin_limit_rejects_invalid_plans(lib):
    f = lib.wsfft_batch_plan_set_spin_limit
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint]
    assert f(None, 5) == BADPLAN
    assert f(ctypes.c_void_p(0x1000), 5) == BADPLAN
