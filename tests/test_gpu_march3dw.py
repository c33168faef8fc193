"""GPU parity of the wavefront 3D passes (k_march3dw: each thread owns a pair
of columns and keeps their last planes in registers; two red-black sweeps
per pass with the zero start / coarse-grid correction in front and the
residual + restriction / residual norm / FP64 accumulation behind), through
the C-ABI.

MGX_M3W sets the smallest level edge that takes them (default 31: every
level above the one-workgroup tail); here it is lowered so that every level from 15 up does, on
grids of one to four 32 x 32 tiles per plane edge with ragged edges and runs
of 2 .. 64 planes.

* against the one-sweep fused passes (MGX_M3W=0): the same arithmetic, the two
  x neighbours summed in another order, so FP64 cycles agree to 1e-13, FP32
  to 1e-6, bf16 state to 2e-2 (one bf16 ulp);
* against the oracle: V-cycle iterates with 1, 2 and 3 sweeps (FP64, 1e-12),
  W- and F-cycles, refinement steps (FP32 2e-5, bf16 3e-2), and solves
  whose fused norm history follows the oracle's.
"""
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


def cycles(monkeypatch, m3w, n, prec, ncyc, seed, nu=2, cycle="V"):
    monkeypatch.setenv("MGX_M3W", str(m3w))
    s = mgx().Solver(n, 3, precision=prec, nu1=nu, nu2=nu, cycle=cycle)
    f = dev(I.normal_rhs(n, 3, seed))
    u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    outs = []
    for _ in range(ncyc):
        s.vcycle(u, f)
        outs.append(host(u).copy())
    s.close()
    return outs


@pytest.mark.parametrize("n,prec,nu", [(63, "f64", 2), (127, "f64", 2), (63, "f64", 3), (63, "f32", 2),
                                       (127, "bf16", 2), (63, "f64", 1)])
def test_wavefront_matches_one_sweep_passes(n, prec, nu, monkeypatch):
    say("3D wavefront vs one-sweep passes n=%d %s nu=%d" % (n, prec, nu))
    a = cycles(monkeypatch, 0, n, prec, 2, 50, nu)
    b = cycles(monkeypatch, 15, n, prec, 2, 50, nu)
    tol = {"f64": 1e-13, "f32": 1e-6, "bf16": 2e-2}[prec]
    for k, (x, y) in enumerate(zip(a, b)):
        d = rel(y, x)
        say("  cycle %d: %s" % (k + 1, "bitwise" if np.array_equal(x, y) else "max rel diff %.3e" % d))
        assert d <= tol


@pytest.mark.parametrize("n,nu,m3w", [(31, 2, 15), (63, 2, 15), (127, 2, 15), (63, 1, 15), (63, 3, 15),
                                      (127, 3, 15), (127, 2, 64)])
def test_wavefront_vcycle_vs_oracle(n, nu, m3w, monkeypatch):
    monkeypatch.setenv("MGX_M3W", str(m3w))
    say("3D wavefront vcycle vs oracle n=%d nu=%d from edge %d" % (n, nu, m3w))
    s = mgx().Solver(n, 3, nu1=nu, nu2=nu)
    f = I.normal_rhs(n, 3, 51)
    u0 = I.normal_rhs(n, 3, 52) * 1e-2
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


@pytest.mark.parametrize("cycle", ["W", "F"])
def test_wavefront_wf_cycles_vs_oracle(cycle, monkeypatch):
    monkeypatch.setenv("MGX_M3W", "15")
    n = 63
    say("3D wavefront %s-cycle vs oracle n=%d" % (cycle, n))
    s = mgx().Solver(n, 3, cycle=cycle)
    f = I.normal_rhs(n, 3, 53)
    u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    s.vcycle(u, dev(f))
    want = O.cycle(np.zeros_like(f), f, kind=cycle)
    d = rel(host(u), want)
    say("  rel diff %.3e" % d)
    assert d <= 1e-12
    s.close()


def test_wavefront_vcycle_255(monkeypatch):
    """The 255 level in wavefront passes (64 tiles per plane, runs of 64
    planes), 127 and below in one-sweep passes."""
    monkeypatch.setenv("MGX_M3W", "255")
    n = 255
    say("3D wavefront vcycle vs oracle n=%d" % n)
    s = mgx().Solver(n, 3)
    f = I.normal_rhs(n, 3, 54)
    u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    s.vcycle(u, dev(f))
    want = O.vcycle(np.zeros_like(f), f)
    d = rel(host(u), want)
    say("  rel diff %.3e" % d)
    assert d <= 1e-12
    s.close()


@pytest.mark.parametrize("n", [63, 127])
def test_wavefront_solve_fused_norm(n, monkeypatch):
    monkeypatch.setenv("MGX_M3W", "15")
    say("3D wavefront fused-norm solve n=%d" % n)
    s = mgx().Solver(n, 3)
    f = I.normal_rhs(n, 3, 55)
    u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    rc, st = s.solve(u, dev(f), rtol=1e-10)
    assert rc == 0
    ref = O.solve(f, tol=1e-10)
    say("  cycles %d (oracle %d)" % (st.cycles, ref.cycles))
    assert abs(st.cycles - ref.cycles) <= 1
    k = min(st.cycles, ref.cycles)
    h = np.array(st.history())[: k + 1]
    tol = 1e-6 + 1e-15 / ref.hist[: k + 1]
    assert np.all(np.abs(h - ref.hist[: k + 1]) <= tol * ref.hist[: k + 1])
    got = host(u)
    assert np.linalg.norm(O.residual(got, f)) / np.linalg.norm(f) <= 1e-10
    s.close()


@pytest.mark.parametrize("n,prec", [(63, "f32"), (63, "bf16"), (127, "f32")])
def test_wavefront_refinement_step_vs_oracle(n, prec, monkeypatch):
    monkeypatch.setenv("MGX_M3W", "15")
    say("3D wavefront refinement step n=%d %s" % (n, prec))
    s = mgx().Solver(n, 3, precision=prec)
    f = I.normal_rhs(n, 3, 56)
    u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    s.vcycle(u, dev(f))
    ref = O.solve_ir(f, prec=O.F32 if prec == "f32" else O.BF16, tol=0.0, maxc=1)
    d = rel(host(u), ref.u)
    say("  rel diff %.3e" % d)
    assert d <= (2e-5 if prec == "f32" else 3e-2)
    s.close()


def test_wavefront_graph_replay(monkeypatch):
    monkeypatch.setenv("MGX_M3W", "15")
    n = 63
    say("3D wavefront graph replay n=%d" % n)
    f = dev(I.normal_rhs(n, 3, 57))
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


@pytest.mark.parametrize("dim,n,prec", [(3, 63, "f64"), (3, 127, "f64"), (2, 255, "f64"), (3, 63, "f32")])
def test_zero_start_solve(dim, n, prec):
    """zero_start=True never reads the u passed in (here filled with NaN):
    the solve equals the one from a zeroed u, history and solution bit for
    bit (the fused 3D path starts its first finest pre-smoothing from zero,
    the others zero u first)."""
    say("zero-start solve dim=%d n=%d %s" % (dim, n, prec))
    f = dev(I.normal_rhs(n, dim, 58))
    out = []
    for zs in (False, True):
        s = mgx().Solver(n, dim, precision=prec, zero_start=zs)
        u = torch.zeros((n,) * dim, dtype=torch.float64, device="cuda")
        if zs:
            u.fill_(float("nan"))
        rc, st = s.solve(u, f, rtol=1e-10)
        assert rc in (0, 2)
        out.append((st.cycles, np.array(st.history()), host(u)))
        s.close()
    (c0, h0, u0), (c1, h1, u1) = out
    assert c0 == c1 and np.array_equal(h0, h1) and np.array_equal(u0, u1)
