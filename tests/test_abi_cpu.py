"""Host-side checks of the C-ABI library that need no GPU: it loads, and it
exports every function include/mg.h declares (and the binding declares)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1210_7774_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "mg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z_0-9]+)\s*\(", txt)))


def test_header_matches_binding():
    assert header_functions() == sorted(_abi.EXPORTS)


@pytest.mark.skipif(not os.path.exists(_abi.LIB_PATH), reason="libmgx.so not built")
def test_library_exports_every_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True, text=True).stdout
    names = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for fn in header_functions():
        assert fn in names, fn
    L = ctypes.CDLL(_abi.LIB_PATH)
    for fn in header_functions():
        assert hasattr(L, fn)


@pytest.mark.skipif(not os.path.exists(_abi.LIB_PATH), reason="libmgx.so not built")
def test_status_strings_and_argument_checks_without_gpu():
    """Pure host paths: status strings, and size queries that reject bad grids
    before touching the device."""
    L = _abi.lib()
    assert L.mg_status_str(0) == b"ok"
    assert L.mg_status_str(-4) == b"non-finite residual"
    g = _abi.Grid()
    g.dim = 2
    g.n[0] = g.n[1] = 100          # not 2^k - 1
    g.n[2] = 1
    nb = ctypes.c_size_t(0)
    o = _abi.Options()
    L.mg_options_default(ctypes.byref(o))
    assert L.mg_workspace_size(ctypes.byref(g), None, ctypes.byref(o), ctypes.byref(nb)) == _abi.MG_ERR_ARG
    g.n[0] = g.n[1] = 127
    assert L.mg_workspace_size(ctypes.byref(g), None, ctypes.byref(o), ctypes.byref(nb)) == _abi.MG_OK
    assert nb.value > 2 * 8 * 63 * 63
    g.dim = 3
    g.n[2] = 127
    op = _abi.Operator(_abi.MG_OP_DIFFUSION, ctypes.c_void_p(16))
    assert L.mg_workspace_size(ctypes.byref(g), ctypes.byref(op), ctypes.byref(o),
                               ctypes.byref(nb)) == _abi.MG_ERR_UNSUPPORTED
    o.nu1 = o.nu2 = 0
    g.dim = 2
    g.n[2] = 1
    assert L.mg_workspace_size(ctypes.byref(g), None, ctypes.byref(o), ctypes.byref(nb)) == _abi.MG_ERR_ARG


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
