"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/hpgmx.h, and rejects bad arguments
before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hpgmx.h")
LIB = os.path.join(ROOT, "paper_2507_11512_amd", "libhpgmx.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hpgmx_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libhpgmx.so is not built; run __graft_entry__.build()")
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["hpgmx_setup_problem", "hpgmx_mg_setup", "hpgmx_gmres_ir_solve",
                     "hpgmx_spmv", "hpgmx_smooth", "hpgmx_vcycle", "hpgmx_restrict_residual",
                     "hpgmx_prolong_add", "hpgmx_destroy", "hpgmx_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_2507_11512_amd import hpgmx
    assert sorted(hpgmx.EXPORTS) == declared_functions()


def test_null_and_invalid_arguments(lib):
    from paper_2507_11512_amd import hpgmx
    h = C.c_void_p()
    f = lib.hpgmx_setup_problem
    f.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]
    f.restype = C.c_int
    assert f(None, None, C.byref(h)) == -1
    for dims in [(0, 4, 4), (4, -1, 4), (2048, 2048, 1024)]:
        d = hpgmx.ProblemDesc(*dims, 0.5)
        assert f(C.byref(d), None, C.byref(h)) == -1
        assert not h.value
    d = hpgmx.ProblemDesc(8, 8, 8, float("nan"))
    assert f(C.byref(d), None, C.byref(h)) == -1
    lib.hpgmx_destroy.argtypes = [C.c_void_p]
    assert lib.hpgmx_destroy(None) == -1
    lib.hpgmx_last_error.argtypes = [C.c_void_p]
    lib.hpgmx_last_error.restype = C.c_char_p
    assert lib.hpgmx_last_error(None) == b"invalid handle"
    for name in ["hpgmx_mg_setup", "hpgmx_spmv", "hpgmx_vcycle", "hpgmx_gmres_ir_solve"]:
        fn = getattr(lib, name)
        fn.restype = C.c_int
    lib.hpgmx_mg_setup.argtypes = [C.c_void_p, C.c_void_p]
    assert lib.hpgmx_mg_setup(None, None) == -1


def test_structs_match_header_layout():
    from paper_2507_11512_amd import hpgmx
    assert C.sizeof(hpgmx.ProblemDesc) == 24
    assert C.sizeof(hpgmx.MgDesc) == 20
    assert C.sizeof(hpgmx.SolveDesc) == 40
    assert C.sizeof(hpgmx.SolveStats) == 48


def test_inputs_module_is_arithmetic_free():
    from paper_2507_11512_amd import inputs
    a = inputs.random_x0(16)
    b = inputs.random_x0(16)
    assert a.shape == (4096,) and (a == b).all() and a.min() >= -1 and a.max() <= 1
