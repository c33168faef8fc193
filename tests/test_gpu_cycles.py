"""W- and F-cycles and full multigrid on the GPU (through the C-ABI) against
the oracle's cycles (oracle.cycle / oracle.fmg / oracle.solve with kind and
fmg), on the same seeded inputs.

Cases span every schedule the host builds: 2D marching and LDS-tiled levels
above the single-workgroup tail, the generic (Jacobi) path, the fused 3D
plane-marching passes, the generic 3D path, 1D hierarchies that fit in the
tail entirely (the tail runs the whole cycle) and one with generic levels
above it, and a 2D hierarchy held entirely by the tail.

Tolerances as for the V-cycle (relative to the max-norm of the reference):
FP64 iterates after one or two cycles or one FMG pass 1e-12, histories 1e-9
(1e-6 for full solves, where the last residuals approach the rounding
floor), FP32 inner cycles 2e-5, bfloat16-state inner cycles 3e-2.
"""
import math

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


def nco(d):
    return 1 if d == 1 else 3


CYCLE_CASES = [
    (2, 255, "W", "rbgs", False),
    (2, 255, "F", "rbgs", False),
    (2, 1023, "W", "rbgs", False),
    (2, 255, "W", "rbgs", True),
    (2, 127, "W", "jacobi", False),
    (2, 127, "F", "jacobi", False),
    (2, 31, "F", "rbgs", False),
    (3, 63, "W", "rbgs", False),
    (3, 63, "F", "rbgs", False),
    (3, 31, "W", "jacobi", False),
    (1, 1023, "W", "rbgs", False),
    (1, 16383, "F", "rbgs", False),
]


@pytest.mark.parametrize("d,n,kind,smoother,vc", CYCLE_CASES)
def test_cycle_fp64(d, n, kind, smoother, vc):
    say("%s-cycle fp64 d=%d n=%d %s vc=%d" % (kind, d, n, smoother, vc))
    M = mgx()
    a = I.lognormal_coef_2d(n, 4100 + n) if vc else None
    s = M.Solver(n, d, a=dev(a) if vc else None, smoother=smoother, ncoarse=nco(d), cycle=kind)
    f = I.normal_rhs(n, d, 4200 + n)
    u0 = I.normal_rhs(n, d, 4300 + n) * 1e-2
    u, fd = dev(u0), dev(f)
    opts = O.Opts(smoother=O.RBGS if smoother == "rbgs" else O.JACOBI, ncoarse=nco(d))
    want = u0.copy()
    for k in range(2):
        s.vcycle(u, fd)
        O.cycle(want, f, a=a, opts=opts, kind=kind)
        r = rel(host(u), want)
        say("  cycle %d: rel %.2e" % (k, r))
        assert r <= 1e-12, k
    s.close()


FMG_CASES = [
    (2, 255, "V", "rbgs", False),
    (2, 255, "W", "rbgs", False),
    (2, 1023, "F", "rbgs", False),
    (2, 255, "F", "rbgs", True),
    (2, 127, "F", "jacobi", False),
    (2, 31, "W", "rbgs", False),
    (3, 63, "F", "rbgs", False),
    (3, 63, "V", "rbgs", False),
    (3, 31, "W", "jacobi", False),
    (1, 1023, "W", "rbgs", False),
    (1, 16383, "V", "rbgs", False),
]


@pytest.mark.parametrize("d,n,kind,smoother,vc", FMG_CASES)
def test_fmg_pass(d, n, kind, smoother, vc):
    """solve() with fmg and max_cycles = 1 runs exactly the FMG pass: its
    iterate against oracle.fmg, its history against the oracle's."""
    say("FMG(%s) d=%d n=%d %s vc=%d" % (kind, d, n, smoother, vc))
    M = mgx()
    a = I.lognormal_coef_2d(n, 4110 + n) if vc else None
    s = M.Solver(n, d, a=dev(a) if vc else None, smoother=smoother, ncoarse=nco(d), cycle=kind, fmg=True,
                 max_cycles=1)
    f = I.normal_rhs(n, d, 4210 + n)
    u0 = I.normal_rhs(n, d, 4310 + n)            # measured as hist[0], then overwritten by the pass
    u = dev(u0)
    rc, st = s.solve(u, dev(f), rtol=0.0, raise_on_error=False)
    assert rc == M._abi.MG_NOT_CONVERGED and st.cycles == 1
    opts = O.Opts(smoother=O.RBGS if smoother == "rbgs" else O.JACOBI, ncoarse=nco(d))
    want = O.fmg(f, a=a, opts=opts, kind=kind)
    r = rel(host(u), want)
    say("  rel %.2e" % r)
    assert r <= 1e-12
    ref = O.solve(f, a=a, opts=opts, tol=0.0, maxc=1, u0=u0, kind=kind, fmg=True)
    assert np.allclose(np.array(st.history()), ref.hist, rtol=1e-9, atol=0)
    s.close()


@pytest.mark.parametrize("kind", ["W", "F"])
def test_fmg_reaches_discretisation_error(kind):
    """One FMG pass on the sine problem: the error against the continuous
    solution is the discretisation error (pi^2 h^2 / 12) max|u| (exactly
    (c_h - 1) max|u| for the discrete operator) to within 2 %."""
    M = mgx()
    for n in (255, 1023):
        h = 1.0 / (n + 1)
        x = I.grid_x(n)
        ue = np.outer(np.sin(math.pi * x), np.sin(math.pi * x))
        ch = math.pi ** 2 * h ** 2 / (4 * math.sin(math.pi * h / 2) ** 2)
        disc = (ch - 1) * np.abs(ue).max()
        s = M.Solver(n, 2, cycle=kind, fmg=True, max_cycles=1)
        u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        s.solve(u, dev(2 * math.pi ** 2 * ue), rtol=0.0, raise_on_error=False)
        err = np.abs(host(u) - ue).max()
        say("  n=%d err/disc %.4f" % (n, err / disc))
        assert abs(err / disc - 1.0) <= 0.02
        s.close()


@pytest.mark.parametrize("d,n,kind,fmg", [(2, 511, "W", False), (2, 511, "F", True), (3, 63, "W", True),
                                          (1, 4095, "F", False)])
def test_solve_cycles_fp64(d, n, kind, fmg):
    say("solve %s fmg=%d d=%d n=%d" % (kind, fmg, d, n))
    M = mgx()
    s = M.Solver(n, d, ncoarse=nco(d), cycle=kind, fmg=fmg)
    f = I.normal_rhs(n, d, 4400 + n)
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    rc, st = s.solve(u, dev(f), rtol=1e-10)
    assert rc == 0
    ref = O.solve(f, tol=1e-10, opts=O.Opts(ncoarse=nco(d)), kind=kind, fmg=fmg)
    assert abs(st.cycles - ref.cycles) <= 1
    k = min(st.cycles, ref.cycles)
    assert np.allclose(np.array(st.history())[: k + 1], ref.hist[: k + 1], rtol=1e-6, atol=0)
    got = host(u)
    assert np.linalg.norm(O.residual(got, f)) / np.linalg.norm(f) <= 1e-10
    s.close()


@pytest.mark.parametrize("d,n,prec,kind", [(2, 255, "f32", "W"), (2, 255, "bf16", "F"), (3, 31, "f32", "F"),
                                           (3, 63, "bf16", "W"), (1, 511, "f32", "W")])
def test_refinement_step_wf(d, n, prec, kind):
    say("refinement step %s d=%d n=%d %s" % (kind, d, n, prec))
    M = mgx()
    s = M.Solver(n, d, precision=prec, ncoarse=nco(d), cycle=kind)
    f = I.normal_rhs(n, d, 4500 + n)
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    s.vcycle(u, dev(f))
    ref = O.solve_ir(f, prec=O.F32 if prec == "f32" else O.BF16, tol=0.0, maxc=1, opts=O.Opts(ncoarse=nco(d)),
                     kind=kind)
    r = rel(host(u), ref.u)
    say("  rel %.2e" % r)
    assert r <= (2e-5 if prec == "f32" else 3e-2)
    # and the refined solve reaches the FP64 tolerance
    u.zero_()
    rc, st = s.solve(u, dev(f), rtol=1e-10)
    assert rc in (0, 2)
    assert np.linalg.norm(O.residual(host(u), f)) / np.linalg.norm(f) <= 1e-10
    s.close()


def test_graph_replay_matches_direct_enqueue():
    """A W-cycle solve with FMG, replayed from a captured cycle, gives the
    same iterate and history as the directly enqueued one; repeated solves
    on the same handle too."""
    M = mgx()
    n = 511
    f = dev(I.normal_rhs(n, 2, 4600))
    outs = []
    for graph in (False, True):
        s = M.Solver(n, 2, cycle="W", fmg=True, use_graph=graph)
        for rep in range(2):
            u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
            rc, st = s.solve(u, f, rtol=1e-11)
            assert rc == 0
            outs.append((host(u), np.array(st.history())))
        s.close()
    for u, h in outs[1:]:
        assert np.array_equal(u, outs[0][0])
        assert np.array_equal(h, outs[0][1])
