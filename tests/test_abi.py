"""CPU-side checks of the C ABI: the library loads, exports every entry
point include/rpyfmm.h declares, and its host-side validation rejects bad
arguments before touching the GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpyfmm.h")
LIB = os.path.join(ROOT, "paper_1711_02976_amd", "librpyfmm.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rpy_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("rpy_plan", "rpy_plan_batched", "rpy_matvec", "rpy_plan_free", "rpy_plan_stats",
                 "rpy_plan_export", "rpy_default_options", "rpy_status_string", "rpy_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (rpy_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_validation_without_gpu():
    import paper_1711_02976_amd as R
    L = R.lib()
    h = C.c_void_p(123)
    # invalid radius, viscosity, eps and counts are rejected before any HIP call
    assert L.rpy_plan(C.byref(h), 10, None, 0.5, 1.0, 1e-6, None) == R.RPY_EINVAL
    assert h.value is None
    assert L.rpy_plan(C.byref(h), 10, C.c_void_p(8), -1.0, 1.0, 1e-6, None) == R.RPY_EINVAL
    assert L.rpy_plan(C.byref(h), 10, C.c_void_p(8), 0.5, 0.0, 1e-6, None) == R.RPY_EINVAL
    assert L.rpy_plan(C.byref(h), 10, C.c_void_p(8), 0.5, 1.0, 0.5, None) == R.RPY_EINVAL
    assert L.rpy_plan(C.byref(h), -1, C.c_void_p(8), 0.5, 1.0, 1e-6, None) == R.RPY_EINVAL
    assert L.rpy_matvec(None, 1, None, None) == R.RPY_EINVAL
    info = R.rpy_sqrt_info_t()
    info.iterations = 77
    assert L.rpy_sqrt_matvec(None, 1, None, None, 1e-6, 10, C.byref(info)) == R.RPY_EINVAL
    assert info.iterations == 0 and b"plan" in L.rpy_last_error()
    assert b"plan" in L.rpy_last_error()
    o = R.make_options(order=99)
    assert L.rpy_plan(C.byref(h), 10, C.c_void_p(8), 0.5, 1.0, 1e-6, C.byref(o)) == R.RPY_EINVAL
    o = R.make_options(max_depth=30)
    assert L.rpy_plan(C.byref(h), 10, C.c_void_p(8), 0.5, 1.0, 1e-6, C.byref(o)) == R.RPY_EINVAL
    o = R.make_options(nrhs=-1)
    assert L.rpy_plan(C.byref(h), 10, C.c_void_p(8), 0.5, 1.0, 1e-6, C.byref(o)) == R.RPY_EINVAL
    assert b"nrhs" in L.rpy_last_error()
    # a caller whose struct ends at `stream` (struct_size = offset of nrhs):
    # the field past it is not read, so its garbage value is not rejected
    o = R.make_options(order=99, nrhs=-7)
    o.struct_size = R.rpy_options.nrhs.offset
    assert L.rpy_plan(C.byref(h), 10, C.c_void_p(8), 0.5, 1.0, 1e-6, C.byref(o)) == R.RPY_EINVAL
    assert b"nrhs" not in L.rpy_last_error()
    o.struct_size = R.rpy_options.stream.offset
    assert L.rpy_plan(C.byref(h), 10, C.c_void_p(8), 0.5, 1.0, 1e-6, C.byref(o)) == R.RPY_EINVAL
    assert b"struct_size" in L.rpy_last_error()
    o = R.make_options(w_direct=-2)
    assert L.rpy_plan(C.byref(h), 10, C.c_void_p(8), 0.5, 1.0, 1e-6, C.byref(o)) == R.RPY_EINVAL
    assert b"w_direct" in L.rpy_last_error()
    assert L.rpy_plan_inject_error(None, 0) == R.RPY_EINVAL
    assert L.rpy_plan_inject_error(None, R.RPY_INJECT_ALLOC) == R.RPY_EINVAL
    o = R.make_options(tune=2)
    assert L.rpy_plan(C.byref(h), 10, C.c_void_p(8), 0.5, 1.0, 1e-6, C.byref(o)) == R.RPY_EINVAL
    assert b"tune" in L.rpy_last_error()
    L.rpy_plan_free(None)  # NULL-safe
    assert L.rpy_status_string(R.RPY_ENONFINITE) == b"non-finite position"
