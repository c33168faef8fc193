"""Batches of independent uneven-size 2D systems through mg_setup_batch /
mg_solve_batch: every system must satisfy the FP64 tolerance by the oracle's
own residual, match a single-system solve of the same problem, and not depend
on the order of the systems in the batch."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def say(*a):
    print(*a, flush=True)


def problems(ns, seed0=7000):
    out = []
    for s, n in enumerate(ns):
        out.append((n, I.lognormal_coef_2d(n, seed0 + s), I.normal_rhs(n, 2, seed0 + 500 + s)))
    return out


@pytest.mark.parametrize("prec", ["f32", "bf16", "f64"])
def test_batch_matches_oracle_and_single(prec):
    import paper_1210_7774_amd as M
    ns = [127, 255, 127, 511, 255]
    say("batch", prec, ns)
    probs = problems(ns)
    coefs = [dev(a) for _, a, _ in probs]
    fs = [dev(f) for _, _, f in probs]
    us = [torch.zeros(n, n, dtype=torch.float64, device="cuda") for n in ns]
    bs = M.BatchSolver(ns, coefs=coefs, precision=prec)
    rc, stats = bs.solve(us, fs, rtol=1e-10)
    assert rc in (0, 2)
    for s, (n, a, f) in enumerate(probs):
        got = us[s].cpu().numpy()
        r = O.residual(got, f, a=a)
        assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-10, s
        assert stats[s].cycles >= 1
        single = M.Solver(n, 2, a=coefs[s], precision=prec)
        u1 = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        rc1, st1 = single.solve(u1, fs[s], rtol=1e-10)
        assert abs(st1.cycles - stats[s].cycles) <= 1, s
        if st1.cycles == stats[s].cycles:
            ref = u1.cpu().numpy()
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), s
        single.close()
    bs.close()


def test_batch_order_invariance_bitwise():
    import paper_1210_7774_amd as M
    ns = [255, 127, 511]
    say("batch order invariance")
    probs = problems(ns, 7100)
    res = {}
    for order in ([0, 1, 2], [2, 0, 1]):
        coefs = [dev(probs[i][1]) for i in order]
        fs = [dev(probs[i][2]) for i in order]
        us = [torch.zeros(ns[i], ns[i], dtype=torch.float64, device="cuda") for i in order]
        bs = M.BatchSolver([ns[i] for i in order], coefs=coefs, precision="f32")
        rc, stats = bs.solve(us, fs, rtol=1e-10)
        assert rc == 0
        for k, i in enumerate(order):
            res.setdefault(i, []).append((stats[k].cycles, us[k].cpu().numpy()))
        bs.close()
    for i, v in res.items():
        assert v[0][0] == v[1][0]
        assert np.array_equal(v[0][1], v[1][1]), i


def test_batch_poisson_fp64_graph():
    import paper_1210_7774_amd as M
    ns = [127, 255, 511, 127]
    say("batch poisson fp64 graph")
    fs_np = [I.normal_rhs(n, 2, 7200 + s) for s, n in enumerate(ns)]
    outs = []
    for g in (False, True):
        us = [torch.zeros(n, n, dtype=torch.float64, device="cuda") for n in ns]
        bs = M.BatchSolver(ns, coefs=None, precision="f64", use_graph=g)
        rc, stats = bs.solve(us, [dev(f) for f in fs_np], rtol=1e-10)
        assert rc == 0
        outs.append([u.cpu().numpy() for u in us])
        for s, f in enumerate(fs_np):
            r = O.residual(outs[-1][s], f)
            assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-10
        bs.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_batch_large_uneven_graph_autotuned():
    """20 systems with sizes from the benchmark's set {127, 255, 511, 1023}
    (1023 included), FP32 cycles in FP64 refinement, autotuned launch shapes
    and a captured graph: every system to 1e-10 by the oracle's residual."""
    import paper_1210_7774_amd as M
    ns = [1023, 127, 511, 255, 1023, 127, 127, 511, 255, 255, 1023, 127, 511, 127, 255, 511, 127, 1023, 255, 127]
    say("batch of %d, n up to 1023" % len(ns))
    probs = problems(ns, 7300)
    coefs = [dev(a) for _, a, _ in probs]
    fs = [dev(f) for _, _, f in probs]
    us = [torch.zeros(n, n, dtype=torch.float64, device="cuda") for n in ns]
    bs = M.BatchSolver(ns, coefs=coefs, precision="f32", use_graph=True)
    bs.autotune(us, fs, reps=2)
    for u in us:
        u.zero_()
    rc, stats = bs.solve(us, fs, rtol=1e-10)
    assert rc in (0, 2)
    for s, (n, a, f) in enumerate(probs):
        r = O.residual(us[s].cpu().numpy(), f, a=a)
        assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-10, s
    bs.close()
