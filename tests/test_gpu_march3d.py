"""GPU parity of the fused 3D plane-marching passes (one red-black sweep per
pass with the zero start / coarse-grid correction in front and the residual +
restriction / residual norm / FP64 accumulation behind), through the C-ABI.
(MGX_M3W=0 keeps every level on these passes.)

* against the unfused 3D path of the same library (half sweeps, separate
  residual, restriction, prolongation and norm kernels; MGX_M3=0): the same
  arithmetic in the same order, so FP64 cycles agree to 1e-13 (FMA
  contraction may differ), FP32 to 1e-6, bf16 state to 2e-2 (one bf16 ulp
  where a contraction moves a value across a rounding boundary);
* against the oracle: V-cycle iterates (FP64, 1e-12), refinement steps
  (FP32 2e-5, bf16 3e-2), solves to 1e-10 by the oracle's own residual, and
  the residual history the fused norm reports (1e-6), on grids that span
  several tiles with ragged edges (tiles are 64 x 8 columns, runs of 8 .. 64
  planes) and with 1, 2 and 3 sweeps.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def one_sweep_passes(monkeypatch):
    """These tests cover the one-sweep passes: keep every level off the
    wavefront passes (their own tests are test_gpu_march3dw.py)."""
    monkeypatch.setenv("MGX_M3W", "0")


def mgx():
    import paper_1210_7774_amd as M
    return M


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def say(*a):
    print(*a, flush=True)


def cycles_with(monkeypatch, m3, n, prec, ncyc, seed, nu=2):
    monkeypatch.setenv("MGX_M3", "1" if m3 else "0")
    monkeypatch.setenv("MGX_RB3_HALF", "1")   # the unfused path: two half sweeps per sweep
    s = mgx().Solver(n, 3, precision=prec, nu1=nu, nu2=nu)
    f = dev(I.normal_rhs(n, 3, seed))
    u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    outs = []
    for _ in range(ncyc):
        s.vcycle(u, f)
        outs.append(host(u).copy())
    s.close()
    return outs


@pytest.mark.parametrize("n,prec", [(63, "f64"), (127, "f64"), (63, "f32"), (127, "bf16"), (255, "f64")])
def test_fused_matches_unfused(n, prec, monkeypatch):
    say("3D fused vs unfused n=%d %s" % (n, prec))
    a = cycles_with(monkeypatch, False, n, prec, 2, 40)
    b = cycles_with(monkeypatch, True, n, prec, 2, 40)
    tol = {"f64": 1e-13, "f32": 1e-6, "bf16": 2e-2}[prec]
    for k, (x, y) in enumerate(zip(a, b)):
        d = rel(y, x)
        say("  cycle %d: %s" % (k + 1, "bitwise" if np.array_equal(x, y) else "max rel diff %.3e" % d))
        assert d <= tol


@pytest.mark.parametrize("n,nu", [(31, 2), (63, 2), (127, 2), (63, 1), (63, 3)])
def test_vcycle_fp64_vs_oracle(n, nu):
    say("3D fused vcycle vs oracle n=%d nu=%d" % (n, nu))
    s = mgx().Solver(n, 3, nu1=nu, nu2=nu)
    f = I.normal_rhs(n, 3, 41)
    u0 = I.normal_rhs(n, 3, 42) * 1e-2
    u = dev(u0)
    fd = dev(f)
    want = u0.copy()
    for k in range(2):
        s.vcycle(u, fd)
        O.vcycle(want, f, opts=O.Opts(nu1=nu, nu2=nu))
        d = rel(host(u), want)
        say("  cycle %d rel diff %.3e" % (k + 1, d))
        assert d <= 1e-12
    s.close()


def test_vcycle_fp64_vs_oracle_255():
    """One cycle at 255^3 (32 x 32 tiles per plane, runs of 32 planes)."""
    n = 255
    say("3D fused vcycle vs oracle n=%d" % n)
    s = mgx().Solver(n, 3)
    f = I.normal_rhs(n, 3, 43)
    u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    s.vcycle(u, dev(f))
    want = O.vcycle(np.zeros_like(f), f)
    d = rel(host(u), want)
    say("  rel diff %.3e" % d)
    assert d <= 1e-12
    s.close()


@pytest.mark.parametrize("n", [63, 127])
def test_solve_fused_norm(n):
    """The last post-sweep of the finest level measures the residual norm:
    the history must follow the oracle's, the solution pass its residual."""
    say("3D fused-norm solve n=%d" % n)
    s = mgx().Solver(n, 3)
    f = I.normal_rhs(n, 3, 44)
    u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    rc, st = s.solve(u, dev(f), rtol=1e-10)
    assert rc == 0
    ref = O.solve(f, tol=1e-10)
    say("  cycles %d (oracle %d)" % (st.cycles, ref.cycles))
    assert abs(st.cycles - ref.cycles) <= 1
    k = min(st.cycles, ref.cycles)
    h = np.array(st.history())[: k + 1]
    # r = f - A u loses digits to cancellation as it nears the rounding floor
    # (about 1e-15 of ||f||), so the relative tolerance widens there
    tol = 1e-6 + 1e-15 / ref.hist[: k + 1]
    assert np.all(np.abs(h - ref.hist[: k + 1]) <= tol * ref.hist[: k + 1])
    got = host(u)
    r = O.residual(got, f)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-10
    if st.cycles == ref.cycles:
        assert rel(got, ref.u) <= 1e-9
    s.close()


@pytest.mark.parametrize("n,prec", [(63, "f32"), (63, "bf16"), (127, "f32"), (127, "bf16")])
def test_refinement_step_vs_oracle(n, prec):
    say("3D fused refinement step n=%d %s" % (n, prec))
    s = mgx().Solver(n, 3, precision=prec)
    f = I.normal_rhs(n, 3, 45)
    u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    s.vcycle(u, dev(f))
    ref = O.solve_ir(f, prec=O.F32 if prec == "f32" else O.BF16, tol=0.0, maxc=1)
    d = rel(host(u), ref.u)
    say("  rel diff %.3e" % d)
    assert d <= (2e-5 if prec == "f32" else 3e-2)
    s.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_refined_solve_fused(prec):
    n = 127
    say("3D fused refined solve n=%d %s" % (n, prec))
    s = mgx().Solver(n, 3, precision=prec)
    f = I.normal_rhs(n, 3, 46)
    u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    rc, st = s.solve(u, dev(f), rtol=1e-10)
    assert rc in (0, 2)
    got = host(u)
    assert np.linalg.norm(O.residual(got, f)) / np.linalg.norm(f) <= 1e-10
    tight = O.solve(f, tol=1e-13)
    assert rel(got, tight.u) <= 1e-8
    s.close()


def test_graph_replay_3d():
    """A captured 3D cycle (fused passes and norm) replays bit for bit like
    stream launches, solve after solve."""
    n = 63
    say("3D graph replay n=%d" % n)
    f = dev(I.normal_rhs(n, 3, 47))
    outs = []
    for g in (False, True):
        s = mgx().Solver(n, 3, use_graph=g)
        for _ in range(3):
            u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
            rc, st = s.solve(u, f, rtol=1e-10)
            assert rc == 0
            outs.append((st.cycles, host(u)))
        s.close()
    for c, o in outs[1:]:
        assert c == outs[0][0] and np.array_equal(o, outs[0][1])
