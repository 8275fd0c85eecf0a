"""The C-ABI library loads on a CPU-only host and exports every function include/pmgfr.h declares
(no compute calls: those need a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmgfr.h")
LIB = os.path.join(ROOT, "paper_1908_03972_amd", "libpmgfr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:pmg_status|int32_t|char\s*\*|const char\s*\*)\s*\**\s*(\w+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for required in ("fr_residual", "fr_element_jacobian", "ejacobi_sweep", "pmg_restrict", "pmg_prolong",
                     "esdirk_stage_solve"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpmgfr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.pmg_abi_version.restype = ctypes.c_int32
    import re
    with open(HEADER) as f:
        version = int(re.search(r"#define PMG_ABI_VERSION (\d+)", f.read()).group(1))
    assert lib.pmg_abi_version() == version
    lib.pmg_last_error.restype = ctypes.c_char_p
    assert lib.pmg_last_error() == b""


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpmgfr.so not built")
def test_argument_errors_are_reported_without_a_gpu():
    from paper_1908_03972_amd import _abi as A
    lib = A.lib()
    h = A.pmg_level()
    assert lib.pmg_level_create(None, ctypes.byref(h)) == A.PMG_E_ARG
    assert b"null" in lib.pmg_last_error()
    d = A.LevelDesc()
    d.dim = 3
    assert lib.pmg_level_create(ctypes.byref(d), ctypes.byref(h)) == A.PMG_E_ARG
    assert lib.fr_residual(None, None, None, None, 0.0, None, None, None) == A.PMG_E_ARG
    assert lib.esdirk_stage_solve(None, 0.0, 0.0, None, None, None, 0, None, None, None, None) == A.PMG_E_ARG


def test_esdirk_tableaux_match_the_oracle():
    """The library's Butcher matrices (a host call, no GPU) equal the oracle's, which the oracle pins
    by the order conditions and L-stability; the two are typed independently from the published
    coefficients."""
    import ctypes as C

    import numpy as np

    from oracle import solver as OS
    from paper_1908_03972_amd import _abi as A
    for scheme, name in ((2, "esdirk2"), (3, "esdirk3"), (4, "esdirk4")):
        ref = OS.esdirk_tableau(name)
        s = ref.shape[0]
        buf = (C.c_double * (s * s))()
        assert A.lib().esdirk_butcher(scheme, buf) == s
        assert np.max(np.abs(np.array(buf[:]).reshape(s, s) - ref)) < 1e-15
    assert A.lib().esdirk_butcher(5, None) == 0


def test_struct_layouts_match_the_header(tmp_path):
    """Every field of the ctypes mirrors in the binding sits at the offset a C compiler gives it
    from include/pmgfr.h, and every struct has the header's size (a field added on one side only
    would shift the rest)."""
    import shutil
    import subprocess
    from paper_1908_03972_amd import _abi as A
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"pmg_level_desc": A.LevelDesc, "pmg_solve_opts": A.SolveOpts, "pmg_solve_stats": A.SolveStats,
               "pmg_nk_opts": A.NkOpts}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "pmgfr.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run([cc, "-std=c99", "-I", inc, "-o", str(exe), str(src)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def _c_class(decl):
    """'ptr', 'i32', 'i64' or 'f64' for one C parameter or return type of the header."""
    d = decl.strip()
    if "*" in d or re.match(r"(const\s+)?(pmg_level|pmg_factors|pmg_batch)\b", d):
        return "ptr"
    t = re.sub(r"\b(const|struct)\b", "", d).split()[0]
    return {"int32_t": "i32", "pmg_status": "i32", "int64_t": "i64", "double": "f64"}[t]


def _py_class(t):
    if t in (ctypes.c_int32,):
        return "i32"
    if t in (ctypes.c_int64,):
        return "i64"
    if t in (ctypes.c_double,):
        return "f64"
    if t in (ctypes.c_void_p, ctypes.c_char_p) or hasattr(t, "_type_") and issubclass(t, ctypes._Pointer):
        return "ptr"
    raise AssertionError(f"unclassified ctypes type {t}")


def test_binding_signatures_match_the_header():
    """Each function the binding declares has the header's arity, and each argument and return value
    the header's kind (pointer or handle, 32- or 64-bit integer, double)."""
    from paper_1908_03972_amd import _abi as A
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    for name, (res, args) in A.SIGNATURES.items():
        m = re.search(r"([\w\s\*]+?)\b" + name + r"\s*\(([^;{}]*)\)\s*;", text)
        assert m, name
        ret = m.group(1).split("\n")[-1]
        params = [p for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
        assert len(params) == len(args), (name, len(params), len(args))
        assert _c_class(ret) == _py_class(res), (name, ret, res)
        for i, (p, a) in enumerate(zip(params, args)):
            assert _c_class(p) == _py_class(a), (name, i, p, a)
