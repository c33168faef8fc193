"""The allocation-free entry point mg_jacobi5_static (its work array is a
static device array of the library) against mg_jacobi5 with a caller work
array, through the C-ABI: bit for bit, on two calls in a row whose second
input is smaller, plus the rejection of sizes above the static maximum."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_static_work_array_matches_caller_work_array():
    from paper_1210_7774_amd import _abi
    L = _abi.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for shape, iters, seed in (((1500, 1700), 11, 81), ((300, 257), 6, 82), ((64, 65), 3, 83)):
        print("jacobi5_static", shape, iters, flush=True)
        x = torch.from_numpy(I.uniform_field(shape, seed)).to("cuda")
        want = torch.empty_like(x)
        work = torch.empty_like(x)
        got = torch.full_like(x, float("nan"))
        rows, cols = shape
        assert L.mg_jacobi5(_p(x), _p(want), _p(work), rows, cols, iters, stream) == _abi.MG_OK
        assert L.mg_jacobi5_static(_p(x), _p(got), rows, cols, iters, stream) == _abi.MG_OK
        torch.cuda.synchronize()
        assert torch.equal(got, want)


def test_static_work_array_limit():
    from paper_1210_7774_amd import _abi
    L = _abi.lib()
    x = torch.zeros(4, 4, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    side = 2049   # 2049^2 doubles exceed the 4,194,304 of the static array
    rc = L.mg_jacobi5_static(_p(x), _p(y), side, side, 5, None)
    assert rc == _abi.MG_ERR_WORKSPACE
    assert b"exceeds" in L.mg_last_error(None)
    # four iterations or fewer need no work array: any size is accepted
    assert L.mg_jacobi5_static(_p(x), _p(y), 4, 4, 4, None) == _abi.MG_OK
    torch.cuda.synchronize()
