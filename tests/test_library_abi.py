"""CPU checks of the C-ABI library: it loads and exports every declared entry
point; the Python binding's structures match the header's layouts."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpgmg.h")
LIB = os.path.join(ROOT, "paper_2304_01728_amd", "libdpgmg.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpg_[a-z_]+)\s*\(", text)))


def _need_lib():
    if not os.path.exists(LIB):
        pytest.skip("libdpgmg.so not built (run python -m paper_2304_01728_amd.build)")


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["dpg_setup", "dpg_assemble", "dpg_build_hierarchy", "dpg_solve", "dpg_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    _need_lib()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (dpg_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        getattr(lib, n)


def test_binding_symbol_list_matches_header():
    from paper_2304_01728_amd import dpgmg
    assert sorted(dpgmg.SYMBOLS) == _declared()


def test_struct_layouts_match_c(tmp_path):
    from paper_2304_01728_amd import dpgmg
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dpgmg.h"\n'
                   'int main(){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(dpg_options),'
                   ' sizeof(dpg_load), sizeof(dpg_info_t), sizeof(dpg_mesh), sizeof(dpg_kstat),'
                   ' offsetof(dpg_options, theta), offsetof(dpg_load, src),'
                   ' offsetof(dpg_options, p_min), offsetof(dpg_info_t, level_p));}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    c = ctypes
    want = [c.sizeof(dpgmg.dpg_options), c.sizeof(dpgmg.dpg_load), c.sizeof(dpgmg.dpg_info_t),
            c.sizeof(dpgmg.dpg_mesh), c.sizeof(dpgmg.dpg_kstat), dpgmg.dpg_options.theta.offset,
            dpgmg.dpg_load.src.offset, dpgmg.dpg_options.p_min.offset,
            dpgmg.dpg_info_t.level_p.offset]
    assert got == want


def test_default_options_without_device():
    _need_lib()
    from paper_2304_01728_amd import dpgmg
    o = dpgmg.dpg_default_options()
    assert (o.precision, o.nu_pre, o.nu_post, o.maxit, o.p_min) == (dpgmg.DPG_FP64, 1, 1, 500, 0)
    assert abs(o.theta - 0.2) < 1e-15
    with pytest.raises(TypeError):
        dpgmg.dpg_default_options(pmin=1)          # not a field: no silent attribute


def test_bad_arguments_rejected_before_any_device_call():
    _need_lib()
    from paper_2304_01728_amd import dpgmg
    L = dpgmg.lib()
    h = ctypes.c_void_p()
    mesh = dpgmg.dpg_mesh(n=4, side=1.0)
    opt = dpgmg.dpg_default_options()
    # p = 0, omega <= 0, n = 0: rejected by argument checks
    assert L.dpg_setup(ctypes.byref(mesh), 0, 1, 1.0, None, None, 0, ctypes.byref(opt),
                       ctypes.byref(h)) == dpgmg.DPG_EINVAL
    assert L.dpg_setup(ctypes.byref(mesh), 2, 1, -1.0, None, None, 0, ctypes.byref(opt),
                       ctypes.byref(h)) == dpgmg.DPG_EINVAL
    bad = dpgmg.dpg_mesh(n=0, side=1.0)
    assert L.dpg_setup(ctypes.byref(bad), 2, 1, 1.0, None, None, 0, ctypes.byref(opt),
                       ctypes.byref(h)) == dpgmg.DPG_EINVAL
    assert L.dpg_assemble(None) == dpgmg.DPG_EINVAL
    assert L.dpg_solve(None, None, 1, 1e-8, None, None, None) == dpgmg.DPG_EINVAL
