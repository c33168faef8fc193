"""Host-side checks of the vector engine (no GPU): kernel formation through
the C-ABI (ve_plan) against the oracle's greedy formation by the paper's
blockable rule, and the generated HIP source of every kernel compiling for
gfx950."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle.vector as V
from paper_1210_7774_amd import _abi
from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.skipif(not os.path.exists(_abi.LIB_PATH), reason="libmgx.so not built")


def as_oracle(instrs):
    conv = lambda x: V.View(*x) if isinstance(x, tuple) else x
    return [(op, conv(out), tuple(conv(x) for x in ins)) for op, out, ins in instrs]


def plan(instrs):
    L = _abi.lib()
    arr = _abi.ve_batch(instrs)
    kof = (ctypes.c_int * max(len(instrs), 1))()
    nk = ctypes.c_int(0)
    assert L.ve_plan(arr, len(instrs), kof, ctypes.byref(nk)) == _abi.VE_OK
    return list(kof)[: len(instrs)], nk.value


def source(instrs, dtypes, k):
    L = _abi.lib()
    arr = _abi.ve_batch(instrs)
    dt = (ctypes.c_int * len(dtypes))(*dtypes)
    need = ctypes.c_size_t(0)
    assert L.ve_kernel_source(arr, len(instrs), dt, len(dtypes), k, None, 0, ctypes.byref(need)) == _abi.VE_OK
    buf = ctypes.create_string_buffer(need.value)
    assert L.ve_kernel_source(arr, len(instrs), dt, len(dtypes), k, buf, need.value,
                              ctypes.byref(need)) == _abi.VE_OK
    return buf.value.decode()


def paper_loop(W=10, H=8):
    R, C = H - 2, W - 2
    v = lambda r0, c0: (0, r0 * W + c0, (R, C), (W, 1))
    work = (1, 0, (R, C), (C, 1))
    t = [(2 + k, 0, (R, C), (C, 1)) for k in range(4)]
    return [("copy", work, (v(1, 1),)), ("add", t[0], (v(0, 1), v(2, 1))), ("add", t[1], (t[0], v(1, 0))),
            ("add", t[2], (t[1], v(1, 2))), ("multiply", t[3], (t[2], 0.2)), ("add", work, (work, t[3])),
            ("copy", v(1, 1), (work,)), ("free", t[0], ()), ("free", t[1], ()), ("free", t[2], ()),
            ("free", t[3], ())]


def test_plan_of_the_paper_loop():
    assert plan(paper_loop()) == ([0, 0, 0, 0, 0, 0, 1, -1, -1, -1, -1], 2)


@pytest.mark.parametrize("seed", range(60))
def test_plan_matches_oracle(seed):
    _, instrs, _ = I.vector_program(seed, reductions=(seed % 4 == 0))
    assert plan(instrs) == V.form_kernels(as_oracle(instrs))


def test_plan_large_views_with_equal_strides():
    """Shifted windows of a large array (the exact lattice test, not the
    small-view enumeration): north / south rows share, interleaved columns
    do not."""
    W, R, C = 4098, 4096, 4096
    v = lambda r0, c0, sc=1, n=C: (0, r0 * W + c0, (R, n), (W, sc))
    t = (1, 0, (R, C), (C, 1))
    assert plan([("add", t, (v(0, 1), v(2, 1))), ("copy", v(1, 1), (t,))]) == ([0, 1], 2)
    ev, od = v(1, 0, 2, 2048), v(1, 1, 2, 2048)
    t2 = (1, 0, (R, 2048), (2048, 1))
    assert plan([("add", ev, (ev, 1.0)), ("multiply", od, (od, ev)), ("copy", t2, (od,))]) == ([0, 0, 0], 1)
    # a view and the same elements reversed: shared, not the same view
    a, r = (0, 0, (W,), (1,)), (0, W - 1, (W,), (-1,))
    assert plan([("negative", a, (a,)), ("copy", (1, 0, (W,), (1,)), (r,))]) == ([0, 1], 2)


def test_launch_argument_caps_split_kernels():
    """More than 64 instructions, or more than 32 constants, in one index
    space: a new kernel (caps the oracle does not have; documented in ve.h)."""
    a, b = (0, 0, (16,), (1,)), (1, 0, (16,), (1,))
    kof, nk = plan([("add", a, (a, b))] * 70)
    assert nk == 2 and kof[:64] == [0] * 64 and kof[64:] == [1] * 6
    kof, nk = plan([("add", a, (a, 1.0))] * 40)
    assert nk == 2 and kof[:32] == [0] * 32 and kof[32:] == [1] * 8


def test_invalid_batches_rejected():
    L = _abi.lib()
    kof = (ctypes.c_int * 2)()
    nk = ctypes.c_int()
    bad_shape = [("add", (0, 0, (4, 4), (4, 1)), ((1, 0, (4, 3), (3, 1)), 1.0))]
    assert L.ve_plan(_abi.ve_batch(bad_shape), 1, kof, ctypes.byref(nk)) == _abi.VE_ERR_ARG
    bad_op = [(77, (0, 0, (4,), (1,)), ((1, 0, (4,), (1,)),))]   # below the user range, not defined
    assert L.ve_plan(_abi.ve_batch(bad_op), 1, kof, ctypes.byref(nk)) == _abi.VE_ERR_ARG
    red = [("add_reduce", (2, 0, (2,), (1,)), ((1, 0, (4,), (1,)),))]   # two-element output
    assert L.ve_plan(_abi.ve_batch(red), 1, kof, ctypes.byref(nk)) == _abi.VE_ERR_ARG


@pytest.mark.slow
def test_generated_kernels_compile_for_gfx950():
    """Every kernel of the paper's loop, of a reduction program and of two
    random programs: the generated source compiles with hipcc for gfx950
    (no contraction, no packed FP32)."""
    progs = [(paper_loop(), [0] * 6)]
    bases, instrs, _ = I.vector_program(3, reductions=True)
    progs.append((instrs, [0] * len(bases)))
    bases, instrs, _ = I.vector_program(7)
    progs.append((instrs, [1] * len(bases)))          # the float build of the same structure
    srcs = []
    for instrs, dts in progs:
        _, nk = plan(instrs)
        srcs += [source(instrs, dts, k) for k in range(nk)]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "k.hip")
        with open(path, "w") as f:
            f.write("#include <hip/hip_runtime.h>\n#define INFINITY __builtin_huge_val()\n")
            seen = set()
            for s in srcs:
                name = s.split("void ", 1)[1].split("(", 1)[0]
                if name not in seen:
                    seen.add(name)
                    f.write(s)
        r = subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-ffp-contract=off", "-c", path,
                            "-o", os.path.join(d, "k.o"), "-Xclang", "-target-feature", "-Xclang",
                            "-packed-fp32-ops"], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
    assert len(seen) >= 5
