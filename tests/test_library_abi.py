"""CPU checks of the boundary: libmgrhip.so loads and exports every entry point
that include/mgr.h declares; the product path has no CPU fallback."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgr.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["mgr_create", "mgr_setup", "mgr_apply", "mgr_apply_transpose", "mgr_solve", "mgr_solve_transpose",
              "mgr_grad_values", "mgr_destroy"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    import paper_2101_11649_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libmgrhip.so not built")
    lib = ctypes.CDLL(P.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert sorted(P.EXPORTED) == declared_symbols()


def test_default_opts_without_gpu():
    import paper_2101_11649_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libmgrhip.so not built")
    o = P.mgr_opts()
    P.lib().mgr_default_opts(ctypes.byref(o))
    assert o.apply_precision == 64 and o.restart == 50 and o.rtol == 1e-8
    assert o.amg.theta == 0.25 and o.amg.max_coarse == 128 and o.amg.seed == 12345


def test_struct_layouts_match_header(tmp_path):
    # compile a probe against include/mgr.h and compare every field's offset
    # and every struct's size with the ctypes binding
    import shutil
    import subprocess
    import paper_2101_11649_amd as P
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = [P.mgr_matrix, P.mgr_level_opts, P.mgr_amg_opts, P.mgr_opts, P.mgr_solve_info]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mgr.h"', 'int main(void) {']
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {" ".join(l.split()[:-1]): int(l.split()[-1]) for l in out if l.strip()}
    for st in structs:
        name = st.__name__
        assert got[f"{name} size"] == ctypes.sizeof(st), name
        for f, _ in st._fields_:
            assert got[f"{name} {f}"] == getattr(st, f).offset, (name, f)


def test_no_cpu_fallback():
    import torch
    import paper_2101_11649_amd as P
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        P.Solver(1, [0, 1], [0], [1.0], [0], [])
