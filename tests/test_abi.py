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


def test_struct_layouts_match_c_compiler(tmp_path):
    # every option/info struct of the header, as gcc lays it out, against the
    # ctypes mirror of the binding (size and the offset of the last field)
    from paper_2202_11599_amd import nysadmm as N
    pairs = [("nys_dense", N.Dense, "data"), ("nys_pcg_opts", N.PcgOpts, "max_restarts"),
             ("nys_pcg_info", N.PcgInfo, "status"), ("nys_problem", N.Problem, "c"),
             ("nys_admm_opts", N.AdmmOpts, "true_res_every"),
             ("nys_admm_state", N.AdmmState, "k"),
             ("nys_admm_info", N.AdmmInfo, "maxiter_solves"),
             ("nys_svm_problem", N.SvmProblem, "C"), ("nys_svm_opts", N.SvmOpts, "factor"),
             ("nys_svm_info", N.SvmInfo, "maxiter_solves")]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "nysadmm.h"', "int main(void){"]
    for cname, _, last in pairs:
        src.append(f'printf("%zu %zu\\n", sizeof({cname}), offsetof({cname}, {last}));')
    src.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for (cname, cls, last), line in zip(pairs, out):
        size, off = map(int, line.split())
        assert ctypes.sizeof(cls) == size, cname
        assert getattr(cls, last).offset == off, cname


def test_option_structs_keep_their_tensors_alive():
    # the structs carry raw device addresses; the binding must hold the
    # tensors (and handles) they point to for as long as the struct lives
    import gc
    import weakref
    import torch
    from paper_2202_11599_amd import nysadmm as N
    om = torch.zeros(3, 8, dtype=torch.float64)
    refs = [weakref.ref(om)]
    o = N.admm_opts(1.0, 3, om)
    s = N.svm_opts(1.0, 3, om)
    del om
    gc.collect()
    assert refs[0]() is not None
    assert o.omega == refs[0]().data_ptr() and s.omega == refs[0]().data_ptr()
    del o, s
    gc.collect()
    assert refs[0]() is None
