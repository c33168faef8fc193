"""GPU parity: the HIP path (through the C-ABI) against the oracle on the same
seeded inputs.

Tolerances (relative to the max-norm of the reference quantity):
  FP64 level operations (one fused pre/post kernel)       1e-13
  FP64 single V-cycle iterate                             1e-12
  FP64 converged solution vs the oracle solved to 1e-13    1e-9
  FP32 inner cycle (one refinement step), vs oracle float  2e-5 of |u|
  bfloat16-state inner cycle, vs oracle bf16 emulation      3e-2 of |u| per step
  every refined solve: final FP64 residual <= tol by the oracle's own residual
The FP64 bound is rounding of a few dozen operations per point (FMA
contraction and association differ from the oracle's plain order); the FP32
bound is ~100 ulp of float; the bf16 bound is one bf16 ulp (2^-8) times the
handful of roundings that differ when an FMA moves a value across a rounding
boundary.
"""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.gpu


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


# ---------------------------------------------------------------- FP64 2D level kernels

@pytest.mark.parametrize("n,G,hb", [(255, 1, 64), (255, 2, 16), (511, 1, 8), (63 + 64, 1, 6)])
def test_fused_pre_kernel_2d(n, G, hb, monkeypatch):
    say("fused pre 2D n=%d G=%d Hb=%d" % (n, G, hb))
    monkeypatch.setenv("MGX_G", str(G))
    monkeypatch.setenv("MGX_HB", str(hb))
    M = mgx()
    s = M.Solver(n, 2)
    u0 = I.normal_rhs(n, 2, 21)
    f = I.normal_rhs(n, 2, 22)
    nc = (n - 1) // 2
    uo = torch.empty(n, n, dtype=torch.float64, device="cuda")
    fc = torch.empty(nc, nc, dtype=torch.float64, device="cuda")
    s.smooth_restrict(dev(u0), dev(f), uo, fc)
    want_u = O.sweep(u0.copy(), f, kind=O.RBGS, nsweeps=2)
    want_fc = O.restrict(O.residual(want_u, f))
    assert rel(host(uo), want_u) <= 1e-13
    # the coarse rhs carries terms of size |u|/h^2: compare on its own scale
    assert rel(host(fc), want_fc) <= 1e-13
    s.close()


@pytest.mark.parametrize("n,G,hb", [(255, 1, 32), (255, 2, 128), (127, 1, 4)])
def test_fused_post_kernel_2d(n, G, hb, monkeypatch):
    say("fused post 2D n=%d G=%d Hb=%d" % (n, G, hb))
    monkeypatch.setenv("MGX_G", str(G))
    monkeypatch.setenv("MGX_HB", str(hb))
    M = mgx()
    s = M.Solver(n, 2)
    nc = (n - 1) // 2
    u0 = I.normal_rhs(n, 2, 23)
    uc = I.normal_rhs(nc, 2, 24)
    f = I.normal_rhs(n, 2, 25)
    uo = torch.empty(n, n, dtype=torch.float64, device="cuda")
    s.correct_smooth(dev(u0), dev(uc), dev(f), uo)
    want = O.prolong_add(uc, u0.copy())
    O.sweep(want, f, kind=O.RBGS, nsweeps=2)
    assert rel(host(uo), want) <= 1e-13
    s.close()


def test_tiling_invariance_bitwise(monkeypatch):
    """The fused kernels recompute their halos, so the result must not depend
    on the strip width or block height, bit for bit."""
    say("tiling invariance")
    n = 511
    f = I.normal_rhs(n, 2, 26)
    outs = []
    for G, hb in ((1, 8), (1, 64), (2, 16), (2, 256)):
        monkeypatch.setenv("MGX_G", str(G))
        monkeypatch.setenv("MGX_HB", str(hb))
        s = mgx().Solver(n, 2)
        u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        fd = dev(f)
        for _ in range(3):
            s.vcycle(u, fd)
        outs.append(host(u))
        s.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_fused_3d_sweep_matches_half_sweeps(prec, monkeypatch):
    """The fused 3D red-black sweep (one pass, plane lag, LDS plane ring)
    against two half sweeps: the same updates in the same sum order, so the
    cycles agree to the last bit up to FMA contraction choices."""
    say("3D fused sweep vs half sweeps", prec)
    monkeypatch.setenv("MGX_M3", "0")   # the one-sweep kernel of the unfused path
    n = 63
    f = I.normal_rhs(n, 3, 27)
    outs = []
    for half in ("1", "0"):
        monkeypatch.setenv("MGX_RB3_HALF", half)
        s = mgx().Solver(n, 3, precision=prec, max_cycles=3)
        u = torch.zeros(n, n, n, dtype=torch.float64, device="cuda")
        rc, st = s.solve(u, dev(f), rtol=1e-14, raise_on_error=False)
        outs.append((st.history()[:4], host(u)))
        s.close()
    (h0, u0), (h1, u1) = outs
    say("bitwise" if np.array_equal(u0, u1) else "max diff %.3e" % np.abs(u0 - u1).max())
    assert np.abs(u0 - u1).max() <= 1e-12 * np.abs(u0).max()
    for a, b in zip(h0[1:], h1[1:]):
        assert abs(a / b - 1.0) <= 1e-9


@pytest.mark.parametrize("prec,vc", [("f64", False), ("f32", True), ("bf16", True)])
def test_tiled_small_levels_match_marching(prec, vc, monkeypatch):
    """Small non-finest 2D levels run as LDS tiles; with the tiles switched
    off they march: the same formulas, so the cycles agree to rounding."""
    say("tiled small levels vs marching", prec, vc)
    n = 1023
    f = I.normal_rhs(n, 2, 28)
    a = I.lognormal_coef_2d(n, 4050) if vc else None
    outs = []
    for tmax in ("0", "511"):
        monkeypatch.setenv("MGX_TILE_MAX", tmax)
        s = mgx().Solver(n, 2, a=dev(a) if vc else None, precision=prec, max_cycles=3)
        u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        rc, st = s.solve(u, dev(f), rtol=1e-14, raise_on_error=False)
        outs.append((st.history()[:4], host(u)))
        s.close()
    (h0, u0), (h1, u1) = outs
    say("bitwise" if np.array_equal(u0, u1) else "max diff %.3e" % np.abs(u0 - u1).max())
    tol = 1e-12 if prec == "f64" else 1e-5
    assert np.abs(u0 - u1).max() <= tol * np.abs(u0).max()
    for a_, b_ in zip(h0[1:], h1[1:]):
        assert abs(a_ / b_ - 1.0) <= (1e-9 if prec == "f64" else 1e-3)


# ---------------------------------------------------------------- FP64 cycles and solves

@pytest.mark.parametrize("d,n,smoother", [(2, 255, "rbgs"), (2, 127, "jacobi"), (3, 31, "rbgs"), (1, 1023, "rbgs"),
                                          (2, 63, "rbgs"), (3, 15, "jacobi")])
def test_vcycle_fp64(d, n, smoother):
    say("vcycle fp64 d=%d n=%d %s" % (d, n, smoother))
    M = mgx()
    nco = 1 if d == 1 else 3
    s = M.Solver(n, d, smoother=smoother, ncoarse=nco)
    f = I.normal_rhs(n, d, 27)
    u0 = I.normal_rhs(n, d, 28) * 1e-2
    u = dev(u0)
    fd = dev(f)
    opts = O.Opts(smoother=O.RBGS if smoother == "rbgs" else O.JACOBI, ncoarse=nco)
    want = u0.copy()
    for k in range(2):
        s.vcycle(u, fd)
        O.vcycle(want, f, opts=opts)
        assert rel(host(u), want) <= 1e-12, k
    s.close()


@pytest.mark.parametrize("d,n", [(2, 255), (2, 1023), (3, 63), (1, 1023)])
def test_solve_fp64(d, n):
    say("solve fp64 d=%d n=%d" % (d, n))
    M = mgx()
    nco = 1 if d == 1 else 3
    s = M.Solver(n, d, ncoarse=nco)
    f = I.normal_rhs(n, d, 29)
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    rc, st = s.solve(u, dev(f), rtol=1e-10)
    assert rc == 0
    ref = O.solve(f, tol=1e-10, opts=O.Opts(ncoarse=nco))
    assert abs(st.cycles - ref.cycles) <= 1
    k = min(st.cycles, ref.cycles)
    h = np.array(st.history())
    assert np.allclose(h[: k + 1], ref.hist[: k + 1], rtol=1e-6, atol=0)
    # same-cycle iterate vs the oracle's (a stop one cycle apart is a
    # reduction-order effect at the tolerance: then compare to a tight solve,
    # whose distance is bounded by the residual reached times ~10)
    got = host(u)
    if st.cycles == ref.cycles:
        assert rel(got, ref.u) <= 1e-9
    else:
        tight = O.solve(f, tol=1e-13, opts=O.Opts(ncoarse=nco))
        assert rel(got, tight.u) <= 1e-8
    r = O.residual(got, f)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-10
    s.close()


def test_solve_varcoef_fp64():
    say("solve varcoef fp64")
    n = 255
    a = I.lognormal_coef_2d(n, 4010)
    f = I.normal_rhs(n, 2, 4510)
    s = mgx().Solver(n, 2, a=dev(a))
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    want = np.zeros_like(f)
    ud, fd = dev(np.zeros_like(f)), dev(f)
    for k in range(2):
        s.vcycle(ud, fd)
        O.vcycle(want, f, a=a)
        assert rel(host(ud), want) <= 1e-12, k
    rc, st = s.solve(u, fd, rtol=1e-10)
    assert rc == 0
    ref = O.solve(f, a=a, tol=1e-10)
    assert abs(st.cycles - ref.cycles) <= 1
    r = O.residual(host(u), f, a=a)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-10
    s.close()


# ---------------------------------------------------------------- mixed precision

@pytest.mark.parametrize("d,n,prec", [(2, 255, "f32"), (2, 255, "bf16"), (3, 31, "f32"), (3, 31, "bf16"),
                                      (1, 511, "f32")])
def test_refinement_step_matches_oracle(d, n, prec):
    say("refinement step d=%d n=%d %s" % (d, n, prec))
    M = mgx()
    nco = 1 if d == 1 else 3
    s = M.Solver(n, d, precision=prec, ncoarse=nco)
    f = I.normal_rhs(n, d, 30)
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    s.vcycle(u, dev(f))
    ref = O.solve_ir(f, prec=O.F32 if prec == "f32" else O.BF16, tol=0.0, maxc=1, opts=O.Opts(ncoarse=nco))
    tol = 2e-5 if prec == "f32" else 3e-2
    assert rel(host(u), ref.u) <= tol
    s.close()


@pytest.mark.parametrize("d,n,prec", [(2, 511, "f32"), (2, 511, "bf16"), (3, 63, "f32"), (3, 63, "bf16")])
def test_refined_solve_reaches_fp64_tolerance(d, n, prec):
    say("refined solve d=%d n=%d %s" % (d, n, prec))
    s = mgx().Solver(n, d, precision=prec)
    f = I.normal_rhs(n, d, 31)
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    rc, st = s.solve(u, dev(f), rtol=1e-10)
    assert rc in (0, 2)
    got = host(u)
    r = O.residual(got, f)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-10
    tight = O.solve(f, tol=1e-13)
    err = rel(got, tight.u)
    say("  cycles", st.cycles, "error vs FP64 oracle", err)
    assert err <= 1e-8
    s.close()


def test_refined_varcoef_solve():
    say("refined varcoef solve")
    n = 255
    a = I.lognormal_coef_2d(n, 4011)
    f = I.normal_rhs(n, 2, 4511)
    s = mgx().Solver(n, 2, a=dev(a), precision="f32")
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    s.vcycle(u, dev(f))
    ref1 = O.solve_ir(f, a=a, prec=O.F32, tol=0.0, maxc=1)
    assert rel(host(u), ref1.u) <= 2e-5
    u.zero_()
    rc, st = s.solve(u, dev(f), rtol=1e-10)
    assert rc == 0
    r = O.residual(host(u), f, a=a)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-10
    s.close()


# ---------------------------------------------------------------- errors and edge cases

def test_error_paths():
    say("error paths")
    M = mgx()
    n = 127
    s = M.Solver(n, 2, max_cycles=1)
    f = I.normal_rhs(n, 2, 32)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    rc, st = s.solve(u, dev(f), rtol=1e-10, raise_on_error=False)
    assert rc == M._abi.MG_NOT_CONVERGED and st.cycles == 1
    fn = f.copy()
    fn[5, 7] = np.nan
    u.zero_()
    rc, st = s.solve(u, dev(fn), rtol=1e-10, raise_on_error=False)
    assert rc == M._abi.MG_ERR_NONFINITE
    # aliasing u and f
    t = dev(f)
    rc, st = s.solve(t, t, rtol=1e-10, raise_on_error=False)
    assert rc == M._abi.MG_ERR_ARG
    s.close()
    with pytest.raises(M.MGError):
        M.Solver(100, 2)
    bad = np.ones((n + 2, n + 2))
    bad[3, 3] = -1.0
    with pytest.raises(M.MGError):
        M.Solver(n, 2, a=dev(bad))


def test_already_converged_and_tiny_grids():
    say("tiny grids")
    M = mgx()
    for n in (1, 3, 7):
        s = M.Solver(n, 2, ncoarse=1 if n == 1 else 3)
        f = I.normal_rhs(n, 2, 33)
        u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        rc, st = s.solve(u, dev(f), rtol=1e-12)
        assert rc == 0
        r = O.residual(host(u), f)
        assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-12
        rc, st = s.solve(u, dev(f), rtol=1e-12)   # starts converged
        assert rc == 0 and st.cycles == 0
        s.close()


def test_graph_replay_matches_stream_launch():
    say("graph replay")
    M = mgx()
    n = 511
    f = dev(I.normal_rhs(n, 2, 34))
    outs = []
    for g in (False, True):
        s = M.Solver(n, 2, use_graph=g)
        for rep in range(2):
            u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
            rc, st = s.solve(u, f, rtol=1e-10)
            assert rc == 0
            outs.append((st.cycles, host(u)))
        s.close()
    for c, o in outs[1:]:
        assert c == outs[0][0] and np.array_equal(o, outs[0][1])
