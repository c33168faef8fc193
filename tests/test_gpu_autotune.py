"""The launch-shape autotuner (mg_autotune / mg_tune_get / mg_tune_set):
whatever shapes it or a caller picks, solves still meet the tolerance by the
oracle's own residual and agree with the untuned solve to rounding."""
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


def relres(u, f, a=None):
    r = O.residual(u, f, a=a) if a is not None else O.residual(u, f)
    return float(np.linalg.norm(r) / np.linalg.norm(f))


@pytest.mark.parametrize("prec,vc", [("f64", False), ("f32", True)])
def test_autotuned_solve_matches_untuned(prec, vc):
    import paper_1210_7774_amd as M
    n = 1023
    say("autotune single", prec, vc)
    f = I.normal_rhs(n, 2, 31)
    a = I.lognormal_coef_2d(n, 4060) if vc else None
    outs = []
    for tune in (False, True):
        s = M.Solver(n, 2, a=dev(a) if vc else None, precision=prec)
        if tune:
            scratch = torch.zeros(n, n, dtype=torch.float64, device="cuda")
            choice = s.autotune(scratch, dev(f), reps=3)
            say("choices", choice)
            # every marching 2D level size is tuned: 1023 down to the tail
            assert 1023 in choice and 511 in choice
            assert not choice[1023][1]  # the finest level never runs as tiles
            assert all(2 <= hb <= 256 for hb, _ in choice.values())
            assert s.tune_get() == choice
        u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        rc, st = s.solve(u, dev(f), rtol=1e-10)
        assert rc == 0
        got = u.cpu().numpy()
        assert relres(got, f, a) <= 1e-10
        outs.append((st.cycles, got))
        s.close()
    (c0, u0), (c1, u1) = outs
    assert abs(c0 - c1) <= 1
    if c0 == c1:
        tol = 1e-10 if prec == "f64" else 1e-6
        assert np.abs(u0 - u1).max() <= tol * np.abs(u0).max()


def test_tune_set_roundtrip_and_forced_shapes():
    import paper_1210_7774_amd as M
    n = 511
    say("tune_set forced shapes")
    f = I.normal_rhs(n, 2, 32)
    s = M.Solver(n, 2)
    # every shape kind: small and large block heights, tiles on a coarse
    # level, and a tile request on the finest level (which marches)
    want = {511: (4, True), 255: (256, True), 127: (6, False)}
    s.tune_set(want)
    assert s.tune_get() == want
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    rc, st = s.solve(u, dev(f), rtol=1e-10)
    assert rc == 0
    assert relres(u.cpu().numpy(), f) <= 1e-10
    with pytest.raises(M.MGError):
        s.tune_set({255: (512, False)})
    with pytest.raises(M.MGError):
        s.tune_set({255: (1, False)})
    s.close()


def test_batch_autotune():
    import paper_1210_7774_amd as M
    ns = [127, 255, 511, 255]
    say("batch autotune", ns)
    coefs_np = [I.lognormal_coef_2d(n, 4100 + s) for s, n in enumerate(ns)]
    fs_np = [I.normal_rhs(n, 2, 4600 + s) for s, n in enumerate(ns)]
    coefs = [dev(a) for a in coefs_np]
    fs = [dev(f) for f in fs_np]
    bs = M.BatchSolver(ns, coefs=coefs, precision="f32")
    us = [torch.zeros(n, n, dtype=torch.float64, device="cuda") for n in ns]
    choice = bs.autotune(us, fs, reps=2)
    say("choices", choice)
    assert {511, 255, 127} <= set(choice)
    for u in us:
        u.zero_()
    rc, stats = bs.solve(us, fs, rtol=1e-10)
    assert rc == 0
    for s, n in enumerate(ns):
        assert relres(us[s].cpu().numpy(), fs_np[s], coefs_np[s]) <= 1e-10, s
    bs.close()


def test_autotune_3d_is_a_no_op():
    import paper_1210_7774_amd as M
    n = 31
    say("autotune 3D")
    f = I.normal_rhs(n, 3, 33)
    s = M.Solver(n, 3)
    u = torch.zeros(n, n, n, dtype=torch.float64, device="cuda")
    assert s.autotune(u, dev(f), reps=2) == {}
    u.zero_()
    rc, st = s.solve(u, dev(f), rtol=1e-10)
    assert rc == 0
    assert relres(u.cpu().numpy(), f) <= 1e-10
    s.close()


def test_autotune_cache(tmp_path):
    import paper_1210_7774_amd as M
    n = 511
    say("autotune cache")
    f = dev(I.normal_rhs(n, 2, 34))
    path = str(tmp_path / "tune.json")
    s = M.Solver(n, 2, precision="f32")
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    first = s.autotune(u, f, reps=2, cache=path)
    s.close()
    # a second solver takes the stored choices without timing them
    s = M.Solver(n, 2, precision="f32")
    assert s.autotune(u, f, reps=2, cache=path) == first
    u.zero_()
    rc, st = s.solve(u, f, rtol=1e-10)
    assert rc == 0
    assert relres(u.cpu().numpy(), f.cpu().numpy()) <= 1e-10
    s.close()
    # another precision is another entry
    s = M.Solver(n, 2, precision="f64")
    s.autotune(u, f, reps=2, cache=path)
    s.close()
    import json
    assert len(json.load(open(path))) == 2


def test_autotune_with_graph_and_learned():
    """Tuning after a graph was captured drops the graph (the work lists
    changed), and a learned handle (finest level generic) tunes its coarser
    marching levels only; both still solve to the tolerance."""
    import paper_1210_7774_amd as M
    import paper_1210_7774_amd.learned as L
    n = 511
    say("autotune with graph / learned")
    f_np = I.normal_rhs(n, 2, 35)
    a_np = I.lognormal_coef_2d(n, 4070)
    f, a = dev(f_np), dev(a_np)
    s = M.Solver(n, 2, use_graph=True)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    rc, st0 = s.solve(u, f, rtol=1e-10)  # captures the graph
    assert rc == 0
    s.tune_set({511: (4, False), 255: (8, False), 127: (32, True)})
    u.zero_()
    rc, st1 = s.solve(u, f, rtol=1e-10)
    assert rc == 0 and abs(st1.cycles - st0.cycles) <= 1
    assert relres(u.cpu().numpy(), f_np) <= 1e-10
    s.close()
    w = L.jacobi_weights(0.8)
    s = M.Solver(n, 2, a=a, smoother="learned", precision="f32", learned=w)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    choice = s.autotune(u, f, reps=2)
    say("learned choices", choice)
    assert 511 not in choice and 255 in choice
    u.zero_()
    rc, st = s.solve(u, f, rtol=1e-8)
    assert rc == 0
    assert relres(u.cpu().numpy(), f_np, a_np) <= 1e-8
    s.close()


def test_unusable_cache_entry_is_a_miss(tmp_path, monkeypatch):
    """A cached entry the handle cannot apply (mg_tune_set fails) is treated
    as a miss: the shapes are tuned again and the entry rewritten."""
    import json

    import paper_1210_7774_amd as M
    n = 511
    say("unusable cache entry")
    f = dev(I.normal_rhs(n, 2, 36))
    path = str(tmp_path / "tune.json")
    s = M.Solver(n, 2)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    first = s.autotune(u, f, reps=2, cache=path)
    key = next(iter(json.load(open(path))))
    calls = []

    def failing_set(obj, choices):
        calls.append(choices)
        raise M.MGError(M._abi.MG_ERR_WORKSPACE, "mg_tune_set")

    monkeypatch.setattr(M, "_tune_set", failing_set)
    again = s.autotune(u, f, reps=2, cache=path)
    assert calls and set(again) == set(first)
    assert key in json.load(open(path))
    u.zero_()
    rc, st = s.solve(u, f, rtol=1e-10)
    assert rc == 0
    s.close()
