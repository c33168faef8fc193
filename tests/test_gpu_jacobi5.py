"""mg_jacobi5 (the paper's fixed-iteration Jacobi benchmark) against the
oracle, bit for bit: both sum centre, up, down, left, right in that order and
scale last, in FP64, so every value must agree exactly."""
import numpy as np
import pytest
import torch

from oracle.jacobi5 import jacobi5 as oracle_jacobi5
from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("shape", [(1, 1), (2, 5), (3, 3), (4, 64), (56, 56), (57, 57), (64, 200), (131, 77),
                                   (1000, 999)])
@pytest.mark.parametrize("iters", [0, 1, 3, 4, 5, 9, 12])
def test_jacobi5_matches_oracle_bitwise(shape, iters):
    import paper_1210_7774_amd as M
    say("jacobi5", shape, iters)
    x = I.uniform_field(shape, 8)
    inp = torch.from_numpy(x).to("cuda")
    out = M.jacobi5(inp, iters=iters)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = oracle_jacobi5(x, iters)
    assert np.array_equal(got, want), np.abs(got - want).max()
    assert np.array_equal(inp.cpu().numpy(), x)  # the input is read only


def test_jacobi5_paper_size():
    """The paper's workload: 7168 x 7168, four iterations (one launch)."""
    import paper_1210_7774_amd as M
    n = 7168
    say("jacobi5 paper size")
    x = I.uniform_field((n, n), 8)
    out = M.jacobi5(torch.from_numpy(x).to("cuda"), iters=4)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle_jacobi5(x, 4))


def test_jacobi5_errors():
    import ctypes

    import paper_1210_7774_amd as M
    from paper_1210_7774_amd import _abi
    L = _abi.lib()
    a = torch.zeros(64, 64, dtype=torch.float64, device="cuda")
    b = torch.zeros(64, 64, dtype=torch.float64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    assert L.mg_jacobi5(p(a), p(b), None, 64, 64, 5, None) == _abi.MG_ERR_ARG  # work needed
    assert L.mg_jacobi5(p(a), p(a), None, 64, 64, 1, None) == _abi.MG_ERR_ARG  # in == out
    assert L.mg_jacobi5(p(a), p(b), p(a), 64, 64, 5, None) == _abi.MG_ERR_ARG  # work == in
    assert L.mg_jacobi5(p(a), p(b), None, 0, 64, 1, None) == _abi.MG_ERR_ARG
    assert L.mg_jacobi5(p(a), p(b), None, 64, 64, -1, None) == _abi.MG_ERR_ARG
    assert L.mg_jacobi5(None, p(b), None, 64, 64, 1, None) == _abi.MG_ERR_ARG
    # the entry point with explicit work and a caller's stream
    x = I.uniform_field((64, 64), 3)
    a.copy_(torch.from_numpy(x))
    w = torch.empty_like(a)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())  # the copy into a is on the default stream
    with torch.cuda.stream(s):
        M.jacobi5(a, iters=7, out=b, work=w, stream=s)
    s.synchronize()
    assert np.array_equal(b.cpu().numpy(), oracle_jacobi5(x, 7))
