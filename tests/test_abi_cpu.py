"""Host-side checks of the C-ABI library that need no GPU: it loads, and it
exports every function include/mg.h declares (and the binding declares)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1210_7774_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(name="mg.h", prefix="mg_"):
    txt = open(os.path.join(ROOT, "include", name)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(%s[a-z_0-9]+)\s*\(" % prefix, txt)))


def test_header_matches_binding():
    assert header_functions() == sorted(_abi.EXPORTS)
    assert header_functions("ve.h", "ve_") == sorted(_abi.VE_EXPORTS)


@pytest.mark.skipif(not os.path.exists(_abi.LIB_PATH), reason="libmgx.so not built")
def test_library_exports_every_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True, text=True).stdout
    names = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for fn in header_functions() + header_functions("ve.h", "ve_"):
        assert fn in names, fn
    L = ctypes.CDLL(_abi.LIB_PATH)
    for fn in header_functions() + header_functions("ve.h", "ve_"):
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


def test_learned_step_rejects_overlapping_output_without_gpu():
    """mg_learned_step checks its arguments before any device call: an output
    that overlaps the iterate, the rhs, the coefficient or the scratch is
    MG_ERR_ARG (the addresses below are never dereferenced)."""
    L = _abi.lib()
    n = 63
    nb = L.mg_learned_scratch_bytes(1, 3)
    V = ctypes.c_void_p
    e, f, a, w, sc = 1 << 20, 1 << 24, 1 << 28, 1 << 30, 1 << 32
    eb = n * n * 4

    def call(out, prec=_abi.MG_P_F32_IR):
        return L.mg_learned_step(V(e), V(out), V(f), V(a), n, prec, V(w), V(sc), nb, None)

    for out in (e, e + eb - 4, f + 8, a + 4 * n, sc + 16, f - eb + 4):
        assert call(out) == _abi.MG_ERR_ARG, hex(out)
    assert call(1 << 34, prec=_abi.MG_P_F64) == _abi.MG_ERR_ARG


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


@pytest.mark.skipif(not os.path.exists(_abi.LIB_PATH), reason="libmgx.so not built")
def test_descriptor_extent_guard():
    """2D levels are addressed through buffer descriptors with 32-bit byte
    counts: a finest FP64 array (with its pitch) or nodal coefficient array
    of 4 GiB or more is rejected before any device work."""
    L = _abi.lib()
    o = _abi.Options()
    L.mg_options_default(ctypes.byref(o))
    nb = ctypes.c_size_t(0)

    def size(n, pitch=0):
        g = _abi.Grid()
        g.dim = 2
        g.n[0] = g.n[1] = n
        g.n[2] = 1
        g.pitch[1] = pitch
        return L.mg_workspace_size(ctypes.byref(g), None, ctypes.byref(o), ctypes.byref(nb))

    assert size(16383) == _abi.MG_OK                  # 2.1 GB per array
    assert size(32767) == _abi.MG_ERR_UNSUPPORTED     # 8.6 GB per array
    assert size(1023, pitch=1 << 20) == _abi.MG_ERR_UNSUPPORTED   # 8.6 GB extent through the pitch
    assert size(1023, pitch=1 << 18) == _abi.MG_OK


def _mon(hist, prec=_abi.MG_P_F64, stall=0.5):
    h = (ctypes.c_double * len(hist))(*hist)
    return _abi.lib().mg_monitor(h, len(hist), prec, stall)


@pytest.mark.skipif(not os.path.exists(_abi.LIB_PATH), reason="libmgx.so not built")
def test_monitor_rules_on_synthetic_histories():
    C, F, D = _abi.MG_MONITOR_CONTINUE, _abi.MG_MONITOR_FALLBACK, _abi.MG_MONITOR_DIVERGED
    bf = _abi.MG_P_F32_BF16_IR
    conv = [1.0, 0.1, 0.01, 1e-3, 1e-4, 1e-5]
    for k in range(1, len(conv) + 1):
        assert _mon(conv[:k]) == C
        assert _mon(conv[:k], bf) == C
    # growth far above the best value so far
    assert _mon([1.0, 0.1, 0.05, 60.0]) == D
    assert _mon([1.0, 0.1, 0.05, 40.0]) == C
    # three rises in a row past the first cycle
    assert _mon([1.0, 0.5, 0.6, 0.7, 0.8]) == D
    assert _mon([1.0, 0.5, 0.6, 0.7]) == C
    assert _mon([1.0, 0.5, 0.6, 0.55, 0.8]) == C
    # a non-finite residual
    assert _mon([1.0, 0.5, float("nan")]) == D
    assert _mon([1.0, float("inf")]) == D
    # bf16 state: the first step may raise the residual (smooth data) ...
    assert _mon([1.0, 112.0], bf) == C
    assert _mon([1.0, 112.0, 0.3], bf) == C
    # ... two consecutive steps after it that each gain less than 2x: fall back
    assert _mon([1.0, 0.02, 0.015, 0.012], bf) == F
    assert _mon([1.0, 0.02, 0.015, 0.006], bf) == C
    assert _mon([1.0, 0.02, 0.015, 0.012], _abi.MG_P_F32_IR) == C   # not for FP32 state
    # the stall ratio is a parameter: demanding 1000x per step falls back at once
    assert _mon(conv[:4], bf, 0.001) == F
    assert _mon(conv[:3], bf, 0.001) == C


@pytest.mark.skipif(not os.path.exists(_abi.LIB_PATH), reason="libmgx.so not built")
def test_cycle_type_and_fmg_options():
    """W / F cycles and the full-multigrid first step: accepted for single
    systems with red-black or Jacobi smoothing, FMG only in FP64; the
    workspace grows by the tail's level-operation schedule."""
    L = _abi.lib()
    g = _abi.Grid()
    g.dim = 2
    g.n[0] = g.n[1] = 255
    g.n[2] = 1
    nb = ctypes.c_size_t(0)

    def size(**kw):
        o = _abi.Options()
        L.mg_options_default(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return L.mg_workspace_size(ctypes.byref(g), None, ctypes.byref(o), ctypes.byref(nb)), nb.value

    rc, v = size()
    assert rc == _abi.MG_OK
    for cyc in (_abi.MG_CYCLE_W, _abi.MG_CYCLE_F):
        rc, w = size(cycle=cyc)
        assert rc == _abi.MG_OK and w > v
        assert size(cycle=cyc, smoother=_abi.MG_SM_JACOBI)[0] == _abi.MG_OK
        assert size(cycle=cyc, precision=_abi.MG_P_F32_IR)[0] == _abi.MG_OK
    assert size(fmg=1)[0] == _abi.MG_OK
    assert size(fmg=1, cycle=_abi.MG_CYCLE_F)[0] == _abi.MG_OK
    assert size(cycle=3)[0] == _abi.MG_ERR_ARG
    assert size(cycle=-1)[0] == _abi.MG_ERR_ARG
    assert size(fmg=2)[0] == _abi.MG_ERR_ARG
    assert size(fmg=1, precision=_abi.MG_P_F32_IR)[0] == _abi.MG_ERR_UNSUPPORTED
    # batches run the V-cycle only
    o = _abi.Options()
    L.mg_options_default(ctypes.byref(o))
    o.cycle = _abi.MG_CYCLE_W
    gs = (_abi.Grid * 2)(g, g)
    assert L.mg_workspace_size_batch(2, gs, None, ctypes.byref(o), ctypes.byref(nb)) == _abi.MG_ERR_UNSUPPORTED
    o.cycle = _abi.MG_CYCLE_V
    assert L.mg_workspace_size_batch(2, gs, None, ctypes.byref(o), ctypes.byref(nb)) == _abi.MG_OK


def test_zero_start_option():
    """zero_start is 0 or 1, for single systems (a batch rejects it)."""
    L = _abi.lib()
    g = _abi.Grid()
    g.dim = 3
    g.n[0] = g.n[1] = g.n[2] = 63
    nb = ctypes.c_size_t(0)
    o = _abi.Options()
    L.mg_options_default(ctypes.byref(o))
    assert o.zero_start == 0
    for v, want in ((1, _abi.MG_OK), (2, _abi.MG_ERR_ARG), (-1, _abi.MG_ERR_ARG)):
        o.zero_start = v
        assert L.mg_workspace_size(ctypes.byref(g), None, ctypes.byref(o), ctypes.byref(nb)) == want
    g.dim = 2
    g.n[2] = 1
    gs = (_abi.Grid * 2)(g, g)
    o.zero_start = 1
    assert L.mg_workspace_size_batch(2, gs, None, ctypes.byref(o), ctypes.byref(nb)) == _abi.MG_ERR_UNSUPPORTED
    o.zero_start = 0
    assert L.mg_workspace_size_batch(2, gs, None, ctypes.byref(o), ctypes.byref(nb)) == _abi.MG_OK
