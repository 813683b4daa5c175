"""CPU checks of the C ABI: the library loads and exports every entry point
that include/nysadmm.h declares, and the binding names match (no compute call
is made: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nysadmm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:nys_status|const\s+char\s*\*|size_t)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libpath():
    from paper_2202_11599_amd import nysadmm
    if not os.path.exists(nysadmm.LIB_PATH):
        from paper_2202_11599_amd import build
        build.build()
    return nysadmm.LIB_PATH


def test_header_declares_the_five_hot_path_calls():
    names = declared_functions()
    for n in ["nys_sketch", "nys_precond_apply", "pcg_solve", "admm_step", "admm_solve"]:
        assert n in names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol(libpath):
    from paper_2202_11599_amd import nysadmm
    assert sorted(nysadmm.EXPORTS) == declared_functions()
    nysadmm.lib()   # binds argtypes for every export without calling any


def test_status_strings_without_gpu(libpath):
    from paper_2202_11599_amd import nysadmm
    assert nysadmm.status_string(0) == "ok"
    assert "invalid" in nysadmm.status_string(1)
    assert "Cholesky" in nysadmm.status_string(3)


def test_struct_layouts_match_header():
    # sizes of the option/info structs as the C compiler lays them out
    from paper_2202_11599_amd import nysadmm as N
    assert ctypes.sizeof(N.Dense) == 40
    assert ctypes.sizeof(N.PcgOpts) == 32
    assert ctypes.sizeof(N.PcgInfo) == 40
