"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (Solver defaults): the 3D Poisson 511^3 and 2D Poisson 4095^2 FP64
solves, and the 511^3 FP32 / bf16-state refinement forms.

An oracle V-cycle at these sizes takes minutes, so the checks are the ones
that hold at any size: the returned solution's relative residual, computed by
the oracle's own residual routine, is at most the tolerance; the library's
residual kernel agrees with the oracle's residual element by element (1e-12
of max|f|: contraction and summation order differ); and the refined
solutions agree with the FP64 solution to the accuracy the tolerance allows.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("d,n,seed", [(3, 511, 3), (2, 4095, 2)])
def test_full_size_fp64_solve(d, n, seed):
    import paper_1210_7774_amd as M
    say("full size FP64 solve d=%d n=%d" % (d, n))
    f_np = I.normal_rhs(n, d, seed)
    f = torch.from_numpy(f_np).cuda()
    s = M.Solver(n, d)
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    rc, st = s.solve(u, f, rtol=1e-10)
    assert rc == 0
    say("  %d cycles, solver rel. residual %.3e" % (st.cycles, st.rel_res))
    got = u.cpu().numpy()
    r_or = O.residual(got, f_np)
    rel = float(np.linalg.norm(r_or) / np.linalg.norm(f_np))
    say("  oracle rel. residual %.3e" % rel)
    assert rel <= 1e-10
    assert abs(rel / st.rel_res - 1.0) <= 1e-3     # two FP64 evaluations of a residual 1e-10 of |f|
    r_gpu = torch.empty_like(u)
    s.residual(u, f, r_gpu)
    diff = float(np.abs(r_gpu.cpu().numpy() - r_or).max() / np.abs(f_np).max())
    say("  residual kernel vs oracle: %.2e of max|f|" % diff)
    assert diff <= 1e-12
    s.close()


def test_full_size_refined_forms_3d():
    import paper_1210_7774_amd as M
    n = 511
    f_np = I.normal_rhs(n, 3, 3)
    f = torch.from_numpy(f_np).cuda()
    ref = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    s = M.Solver(n, 3)
    assert s.solve(ref, f, rtol=1e-10)[0] == 0
    s.close()
    ref_np = ref.cpu().numpy()
    for prec in ("f32", "bf16"):
        say("full size refined form %s" % prec)
        s = M.Solver(n, 3, precision=prec)
        u = torch.zeros_like(ref)
        rc, st = s.solve(u, f, rtol=1e-10)
        assert rc in (0, 2)
        got = u.cpu().numpy()
        rel = float(np.linalg.norm(O.residual(got, f_np)) / np.linalg.norm(f_np))
        say("  %d steps, oracle rel. residual %.3e" % (st.cycles, rel))
        assert rel <= 1e-10
        # both solutions are within rtol of the discrete solution in the
        # residual norm; their difference is a small multiple of that
        assert np.abs(got - ref_np).max() <= 1e-7 * np.abs(ref_np).max()
        s.close()
