"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, the ctypes structures match the C
layout, and argument validation fails before touching the device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrf.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:mrf_status|const char \*)\s*(mrf_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def m():
    import paper_1810_01967_amd as pkg
    pkg.lib()
    return pkg


def test_header_declares_expected_entry_points():
    names = _declared()
    for n in ("mrf_dict_build", "mrf_match", "mrf_ipg_step", "mrf_ipg_solve"):
        assert n in names


def test_library_exports_every_declared_symbol(m):
    out = subprocess.run(["nm", "-D", "--defined-only", m.mrf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (mrf_\w+)$", out, re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    assert set(m.mrf.EXPORTS) == set(_declared())


def test_binding_declares_every_argument(m):
    """Every entry point the binding calls has ctypes argtypes whose count
    matches the header: without them ctypes passes a Python int as a 32-bit
    C int, which silently truncates 64-bit device pointers and sizes."""
    text = open(HEADER).read()
    L = m.lib()
    for name, params in re.findall(r"^\s*(?:mrf_status|const char \*)\s*(mrf_\w+)\s*\(([^;]*?)\);", text, re.M | re.S):
        nparam = 0 if params.strip() in ("", "void") else params.count(",") + 1
        at = getattr(L, name).argtypes
        if nparam == 0:
            continue
        assert at is not None, f"{name}: no argtypes"
        assert len(at) == nparam, f"{name}: {len(at)} argtypes, header has {nparam} parameters"


def test_struct_layout_matches_header(m, tmp_path):
    """Compile the header with the host C compiler and compare sizeof/offsetof
    with the ctypes mirrors of the binding."""
    structs = {"mrf_dict_desc": m.mrf.DictDesc, "mrf_dict_info": m.mrf.DictInfo,
               "mrf_match_opts": m.mrf.MatchOpts, "mrf_match_stats": m.mrf.MatchStats,
               "mrf_op": m.mrf.Op, "mrf_step_stats": m.mrf.StepStats,
               "mrf_solve_opts": m.mrf.SolveOpts, "mrf_solve_stats": m.mrf.SolveStats,
               "mrf_train_opts": m.mrf.TrainOpts, "mrf_train_stats": m.mrf.TrainStats,
               "mrf_tree_info": m.mrf.TreeInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, f"{cname}.{fname}"


def test_validation_fails_before_device_work(m):
    L = m.lib()
    assert L.mrf_dict_build(None, None, None) == m.mrf.MRF_E_INVAL
    assert b"null" in L.mrf_last_error()
    h = ctypes.c_void_p()
    atoms = np.ones((4, 3))
    params = np.zeros(4)
    desc = m.mrf.DictDesc(0, 3, 1, 0, atoms.ctypes.data, 0, params.ctypes.data, None, 0)
    assert L.mrf_dict_build(ctypes.byref(desc), None, ctypes.byref(h)) == m.mrf.MRF_E_INVAL
    desc = m.mrf.DictDesc(4, 3, 1, 0, atoms.ctypes.data, 0, params.ctypes.data, None, 0x100)
    assert L.mrf_dict_build(ctypes.byref(desc), None, ctypes.byref(h)) == m.mrf.MRF_E_INVAL
    gd = np.array([3], dtype=np.int32)      # product 3 != d = 4
    desc = m.mrf.DictDesc(4, 3, 1, 0, atoms.ctypes.data, 0, params.ctypes.data, gd.ctypes.data, 0)
    assert L.mrf_dict_build(ctypes.byref(desc), None, ctypes.byref(h)) == m.mrf.MRF_E_INVAL
    assert b"grid_dims" in L.mrf_last_error()
    opts = m.mrf.MatchOpts(0, 0, 8, 0, None, 3, 0.98, 0, 0.0, 0)
    assert L.mrf_match(None, ctypes.byref(opts), 1, None, 0, 0, None, None, None, None, None, None,
                       None, None) == m.mrf.MRF_E_INVAL
    bad = m.mrf.Op(48, 64, 10, 1, 0, None, None, None)      # 48 is not a power of two
    assert L.mrf_op_forward(ctypes.byref(bad), None, None, None, None, None) == m.mrf.MRF_E_INVAL
    assert L.mrf_quantize_rows(None, 1, 4, 4, 1, None, 4, None, None) == m.mrf.MRF_E_INVAL
    assert L.mrf_dict_destroy(None) == m.mrf.MRF_OK
    assert m.mrf_version().startswith("mrf-mi355x")
