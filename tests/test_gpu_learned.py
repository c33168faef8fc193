"""Learned smoother on the GPU against the FP64 oracle (oracle/learned.py):
network forward pass (bf16 weights and activations, FP32 accumulation)
element by element, energy-norm loss and weight gradient, one Adam step, the
pair gather, the scaled residual, the solver with the exact special-case
network (damped Jacobi) cycle by cycle, and the fallback rules."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import oracle.learned as LN
from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def rel_l2(got, want):
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


@pytest.mark.parametrize("B,H,W", [(1, 16, 16), (3, 37, 45), (2, 5, 70)])
def test_forward_matches_oracle(B, H, W):
    import paper_1210_7774_amd.learned as L
    say("learned forward", B, H, W)
    rng = np.random.default_rng(100 + H)
    s = f32(rng.standard_normal((B, H, W)))
    w = I.he_normal_weights(11).astype(np.float64)
    got = L.apply(dev(s, torch.float32), dev(w, torch.float32)).cpu().numpy().astype(np.float64)
    want = LN.forward(s, w, bf16_emul=True)
    # FP32 accumulation order only; a bf16 activation rounding may flip by one
    # ulp (2^-8 relative) where the FP32 sums straddle a rounding boundary
    assert rel_l2(got, want) <= 1e-3
    assert np.abs(got - want).max() <= 1e-2 * np.abs(want).max()


def test_forward_special_cases():
    import paper_1210_7774_amd.learned as L
    say("learned special cases")
    rng = np.random.default_rng(5)
    s = f32(rng.standard_normal((2, 33, 20)))
    st = dev(s, torch.float32)
    # omega * identity network: exactly omega * bf16(s)
    y = L.apply(st, dev(LN.omega_identity(0.5), torch.float32)).cpu().numpy()
    assert np.array_equal(y.astype(np.float64), 0.5 * LN.bf16(s))
    # zero weights: zero output
    y0 = L.apply(st, torch.zeros(LN.NWEIGHTS, dtype=torch.float32, device="cuda")).cpu().numpy()
    assert np.all(y0 == 0.0)
    # positive homogeneity is exact for powers of two
    w = dev(I.he_normal_weights(12), torch.float32)
    y1 = L.apply(st, w).cpu().numpy()
    y8 = L.apply(dev(8.0 * s, torch.float32), w).cpu().numpy()
    assert np.array_equal(8.0 * y1, y8)


def rand_pairs(B, P, seed):
    rng = np.random.default_rng(seed)
    s = f32(rng.standard_normal((B, P, P)))
    e = f32(rng.standard_normal((B, P, P)))
    a = f32(np.exp(0.7 * rng.standard_normal((B, P, P))))
    return s, e, a


@pytest.mark.parametrize("B,P,border", [(4, 40, 5), (2, 16, 2), (32, 64, 5)])
def test_loss_and_gradient_match_oracle(B, P, border):
    import paper_1210_7774_amd.learned as L
    say("learned loss/grad", B, P, border)
    s, e, a = rand_pairs(B, P, 200 + P)
    w = I.he_normal_weights(13).astype(np.float64)
    loss, g = L.loss_grad(dev(s, torch.float32), dev(e, torch.float32), dev(a, torch.float32),
                          dev(w, torch.float32), border=border)
    g = g.cpu().numpy().astype(np.float64)
    want_L, want_g = LN.loss_and_grad(s, e, a, w, border=border, bf16_emul=True)
    assert abs(loss - want_L) <= 1e-4 * want_L
    # gradient signals are stored in bf16 on the GPU (FP64 in the oracle)
    assert rel_l2(g, want_g) <= 2e-2
    cos = float(g @ want_g / (np.linalg.norm(g) * np.linalg.norm(want_g)))
    assert cos >= 0.999
    # each layer separately, so no layer hides behind a larger one
    k = 0
    for co, ci in LN.SHAPES:
        m = co * ci * 9
        assert rel_l2(g[k:k + m], want_g[k:k + m]) <= 3e-2, (co, ci)
        k += m


def test_one_adam_step_matches_oracle():
    import paper_1210_7774_amd.learned as L
    say("learned adam step")
    B, P = 8, 32
    s, e, a = rand_pairs(B, P, 300)
    w0 = I.he_normal_weights(14)
    wt = dev(w0)
    _, g = L.loss_grad(dev(s, torch.float32), dev(e, torch.float32), dev(a, torch.float32), wt, border=5)
    g = g.cpu().numpy().astype(np.float64)
    res = L.train(dev(s, torch.float32), dev(e, torch.float32), dev(a, torch.float32), wt, epochs=1, batch=B,
                  border=5, lr=1e-3)
    assert res.steps == 1
    want, _, _ = LN.adam_step(w0.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1)
    got = wt.cpu().numpy().astype(np.float64)
    # the training batch visits the pairs in another order than loss_grad did:
    # only the rounding of the gradient differs, which moves an Adam step
    # only where |g| is near eps
    big = np.abs(g) > 1e-5
    assert np.abs(got - want)[big].max() <= 2e-6
    assert np.abs(got - want).max() <= 2.1e-3
    assert np.isfinite(res.loss_hist[0])


def test_crop_gather_is_exact():
    import paper_1210_7774_amd.learned as L
    say("learned crop")
    n, P = 40, 8
    rng = np.random.default_rng(400)
    s, us, uk = (rng.standard_normal((n, n)) for _ in range(3))
    a = np.exp(rng.standard_normal((n + 2, n + 2)))
    off = np.array([[0, 0], [n - P, n - P], [3, 17], [n - P + 1, 0]], dtype=np.int32)
    S, E, A = L.crop(dev(s), dev(us), dev(uk), dev(a), dev(off), P)
    S, E, A = S.cpu().numpy(), E.cpu().numpy(), A.cpu().numpy()
    for c in range(3):
        y, x = off[c]
        assert np.array_equal(S[c], s[y:y + P, x:x + P].astype(np.float32))
        assert np.array_equal(E[c], (us - uk)[y:y + P, x:x + P].astype(np.float32))
        assert np.array_equal(A[c], a[y + 1:y + 1 + P, x + 1:x + 1 + P].astype(np.float32))
    # a crop outside the grid is NaN, not a read out of bounds
    assert np.all(np.isnan(S[3])) and np.all(np.isnan(E[3])) and np.all(np.isnan(A[3]))


def test_scaled_residual_matches_oracle():
    import paper_1210_7774_amd as M
    say("scaled residual")
    n = 63
    a = I.lognormal_coef_2d(n, 4040)
    f = I.normal_rhs(n, 2, 4540)
    u = I.normal_rhs(n, 2, 4541) * 1e-3
    sol = M.Solver(n, 2, a=dev(a))
    got = sol.scaled_residual(dev(u), dev(f)).cpu().numpy()
    want = LN.scaled_residual(u, f, a, 1.0 / (n + 1))
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    sol.close()


@pytest.mark.parametrize("prec,n", [("f32", 63), ("bf16", 63), ("f32", 255)])
def test_identity_network_solver_follows_oracle(prec, n):
    """N = omega * identity makes the learned step damped Jacobi on bf16(s):
    the GPU solve (FP32 inner cycles in FP64 refinement) must follow the FP64
    oracle's learned V-cycle cycle by cycle and reach 1e-10.  At n = 255 the
    learned finest level sits above a row-marching level (127)."""
    import paper_1210_7774_amd as M
    say("learned identity solver", prec, n)
    a = I.lognormal_coef_2d(n, 4030)
    f = I.normal_rhs(n, 2, 4530)
    w = LN.omega_identity(0.75)
    u = np.zeros_like(f)
    want = [1.0]
    for _ in range(4):
        u = LN.learned_vcycle(u, f, a, w, bf16_emul=True)
        want.append(np.linalg.norm(O.residual(u, f, a=a)) / np.linalg.norm(f))
    sol = M.Solver(n, 2, a=dev(a), smoother="learned", precision=prec, learned=dev(w, torch.float32))
    ud = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    rc, st = sol.solve(ud, dev(f), rtol=1e-10)
    assert rc == 0 and st.fell_back == 0, (rc, st.history())
    got = st.history()
    # FP32 inner cycles follow the FP64 cycle to a few percent; bf16-stored
    # inner state (8-bit significand) perturbs each correction by up to ~1e-2
    # relative, which shows in the per-cycle residual by up to a third
    tol = 0.05 if prec == "f32" else 0.35
    for k in range(1, 5):
        assert abs(got[k] / want[k] - 1.0) <= tol, (k, got[:6], want)
    r = O.residual(ud.cpu().numpy(), f, a=a)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-10
    sol.close()


@pytest.mark.parametrize("kind,n", [("negated", 127), ("nan", 127), ("negated", 511), ("nan", 511)])
def test_learned_fallback(kind, n):
    """A network that makes cycles diverge (negated damping) or produces NaN
    hands the solve to red-black Gauss-Seidel: status MG_FELL_BACK and the
    plain tolerance reached."""
    import paper_1210_7774_amd as M
    say("learned fallback", kind, n)
    a = I.lognormal_coef_2d(n, 4031)
    f = I.normal_rhs(n, 2, 4531)
    w = LN.omega_identity(-0.75) if kind == "negated" else np.full(LN.NWEIGHTS, np.nan)
    sol = M.Solver(n, 2, a=dev(a), smoother="learned", precision="f32", learned=dev(w, torch.float32))
    ud = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    rc, st = sol.solve(ud, dev(f), rtol=1e-10)
    assert rc == M._abi.MG_FELL_BACK and st.fell_back == 1, (rc, st.history()[:8])
    r = O.residual(ud.cpu().numpy(), f, a=a)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-10
    # the next solve on the same handle starts with the learned smoother again
    ud.zero_()
    rc2, st2 = sol.solve(ud, dev(f), rtol=1e-10)
    assert rc2 == M._abi.MG_FELL_BACK
    sol.close()


def test_pairs_and_short_training_reduce_loss():
    import paper_1210_7774_amd.learned as L
    say("learned pairs + training")
    n = 127
    probs = [(I.lognormal_coef_2d(n, 6000 + i), I.normal_rhs(n, 2, 6100 + i)) for i in range(2)]
    S, E, A = L.make_pairs(probs, cycles=4, crops=8, patch=32, seed=7200)
    assert S.shape == (128, 32, 32)
    assert torch.isfinite(S).all() and torch.isfinite(E).all() and torch.isfinite(A).all()
    # pair 0 against the oracle: s_0 = D^-1 f (u_0 = 0), e_0 = u*
    off = I.crop_offsets(n, 32, 8, 7200)
    a0, f0 = probs[0]
    s0 = LN.scaled_residual(np.zeros_like(f0), f0, a0, 1.0 / (n + 1))
    y, x = off[0]
    assert np.abs(S[0].cpu().numpy() - s0[y:y + 32, x:x + 32]).max() <= 1e-6 * np.abs(s0).max()
    # pair 8 (cycle 0, post-smoother input): u after a V(2,0) cycle from 0
    u1 = np.zeros_like(f0)
    O.vcycle(u1, f0, a=a0, opts=O.Opts(nu1=2, nu2=0))
    s1 = LN.scaled_residual(u1, f0, a0, 1.0 / (n + 1))
    ustar = O.solve(f0, a=a0, tol=1e-12, maxc=200).u
    y, x = I.crop_offsets(n, 32, 8, 7201)[0]
    assert np.abs(S[8].cpu().numpy() - s1[y:y + 32, x:x + 32]).max() <= 1e-6 * np.abs(s1).max()
    e1 = (ustar - u1)[y:y + 32, x:x + 32]
    assert np.abs(E[8].cpu().numpy() - e1).max() <= 1e-5 * np.abs(e1).max()
    w = L.initial_weights(7000)
    res = L.train(S, E, A, w, epochs=6, batch=16, border=5, lr=1e-3)
    say("loss per epoch", res.loss_hist)
    assert res.steps == 6 * 8
    assert all(np.isfinite(res.loss_hist))
    assert res.loss_hist[-1] < res.loss_hist[0]


def test_fused_step_matches_layer_by_layer():
    """The solver's fused learned step (one kernel, LDS-resident maps, every
    layer on MFMA) against the one-kernel-per-layer chain (VALU for the
    1-channel layers) on the same network: the same bf16 products summed in
    FP32 in another order, so the iterates agree to FP32 rounding amplified by
    the occasional bf16 rounding flip."""
    import os
    import paper_1210_7774_amd as M
    say("learned fused vs layer-by-layer")
    n = 255
    a = dev(I.lognormal_coef_2d(n, 4032))
    f = dev(I.normal_rhs(n, 2, 4532))
    w = LN.omega_identity(0.6) + 0.02 * I.he_normal_weights(15).astype(np.float64)
    wt = dev(w, torch.float32)
    outs = []
    for unfused in ("0", "1"):
        os.environ["MGX_LEARNED_UNFUSED"] = unfused
        try:
            sol = M.Solver(n, 2, a=a, smoother="learned", precision="f32", learned=wt, max_cycles=3)
        finally:
            os.environ.pop("MGX_LEARNED_UNFUSED", None)
        u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        rc, st = sol.solve(u, f, rtol=1e-14, raise_on_error=False)
        outs.append((rc, st.history()[:4], u.cpu().numpy()))
        sol.close()
    (rc0, h0, u0), (rc1, h1, u1) = outs
    say("histories", h0, h1, "bitwise" if np.array_equal(u0, u1) else "differ")
    assert rc0 == rc1
    for k in range(1, 4):
        assert abs(h0[k] / h1[k] - 1.0) <= 1e-2, (h0, h1)
    assert np.abs(u0 - u1).max() <= 1e-4 * np.abs(u1).max()


def test_jacobi_weights_match_oracle():
    import paper_1210_7774_amd.learned as L
    assert np.array_equal(L.jacobi_weights(0.8).cpu().numpy(), LN.omega_identity(0.8).astype(np.float32))


def test_trained_network_gain_over_plain():
    """Train on pairs from the plain solver's cycles (small problems), then
    compare on a held-out problem: the trained network must lower the
    held-out patch loss below its starting point (the damped-Jacobi network)
    and solve to 1e-8 without falling back, in no more cycles than plain
    red-black Gauss-Seidel and with a smaller mean convergence factor (as
    measured on an MI355X: 11 cycles against 12, rho 0.178 against 0.205);
    the time, printed, is not asserted (a learned step costs about four
    fused red-black sweeps, so fewer cycles need not mean less time)."""
    import time
    import paper_1210_7774_amd as M
    import paper_1210_7774_amd.learned as L
    say("learned gain")
    n = 255
    train = [(I.lognormal_coef_2d(n, 6000 + i), I.normal_rhs(n, 2, 6100 + i)) for i in range(6)]
    S, E, A = L.make_pairs(train, cycles=10, crops=12, patch=64, seed=7200, stages=("pre", "post", "noise"))
    held = [(I.lognormal_coef_2d(n, 5000), I.normal_rhs(n, 2, 5001))]
    Sh, Eh, Ah = L.make_pairs(held, cycles=10, crops=16, patch=64, seed=9200, stages=("pre", "post"))
    w0 = L.jacobi_start(0.8, 7001, 0.01)
    w = w0.clone()
    res = L.train(S, E, A, w, epochs=10, batch=32, border=5, lr=1e-4)
    loss0, _ = L.loss_grad(Sh, Eh, Ah, w0)
    loss1, _ = L.loss_grad(Sh, Eh, Ah, w)
    say("held-out loss: start %.4f trained %.4f (train loss %s)" % (loss0, loss1, res.loss_hist))
    assert loss1 < loss0
    a = dev(held[0][0])
    f = dev(held[0][1])
    out = {}
    for name, kw in (("plain", {}), ("learned", dict(smoother="learned", learned=w))):
        sol = M.Solver(n, 2, a=a, precision="f32", **kw)
        u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        rc, st = sol.solve(u, f, rtol=1e-8)
        torch.cuda.synchronize()
        t = time.time()
        u.zero_()
        rc, st = sol.solve(u, f, rtol=1e-8)
        torch.cuda.synchronize()
        out[name] = (rc, st.cycles, st.rho_avg, (time.time() - t) * 1e3, st.fell_back)
        r = O.residual(u.cpu().numpy(), held[0][1], a=held[0][0])
        assert np.linalg.norm(r) / np.linalg.norm(held[0][1]) <= 1e-8
        sol.close()
    say("plain   rc %d cycles %d rho %.4f %.3f ms fell_back %d" % out["plain"])
    say("learned rc %d cycles %d rho %.4f %.3f ms fell_back %d" % out["learned"])
    assert out["learned"][0] == 0 and out["learned"][4] == 0
    assert out["learned"][1] <= out["plain"][1]
    assert out["learned"][2] < out["plain"][2]


def test_learned_error_paths():
    """Bad arguments come back as errors, never as out-of-range reads: a
    visiting order outside [0, npairs) is rejected before any training; a
    learned solver needs weights, 2D, diffusion and a refinement precision."""
    import paper_1210_7774_amd as M
    import paper_1210_7774_amd.learned as L
    say("learned error paths")
    B, P = 4, 16
    s, e, a = rand_pairs(B, P, 500)
    S, E, A = (dev(x, torch.float32) for x in (s, e, a))
    w = L.initial_weights(1)
    w0 = w.clone()
    work = L.scratch(B, P)
    bad = torch.tensor([0, 1, 2, 7], dtype=torch.int32, device="cuda")  # 7 >= npairs
    o = M._abi.TrainOptions(1, B, P, 5, 1e-3, 0.9, 0.999, 1e-8)
    rc = M._abi.lib().mg_learned_train(L._p(S), L._p(E), L._p(A), B, L._p(bad), ctypes.byref(o), L._p(w), None,
                                       None, L._p(work), work.numel(), L._stream())
    assert rc == M._abi.MG_ERR_ARG
    assert torch.equal(w, w0)  # nothing was trained
    rc = M._abi.lib().mg_learned_loss_grad(L._p(S), L._p(E), L._p(A), B, P, 8, L._p(w), ctypes.byref(ctypes.c_double()),
                                           L._p(torch.empty_like(w)), L._p(work), work.numel(), L._stream())
    assert rc == M._abi.MG_ERR_ARG  # 2 * border >= P
    rc = M._abi.lib().mg_learned_loss_grad(L._p(S), L._p(E), L._p(A), B, P, 5, L._p(w), ctypes.byref(ctypes.c_double()),
                                           L._p(torch.empty_like(w)), L._p(work), 16, L._stream())
    assert rc == M._abi.MG_ERR_WORKSPACE
    n = 63
    ad = dev(I.lognormal_coef_2d(n, 1))
    with pytest.raises(M.MGError):
        M.Solver(n, 2, a=ad, smoother="learned", precision="f64", learned=w)   # FP64: unsupported
    with pytest.raises(M.MGError):
        M.Solver(n, 2, smoother="learned", precision="f32", learned=w)          # Poisson: unsupported
    with pytest.raises(M.MGError):
        M.Solver(n, 2, a=ad, smoother="learned", precision="f32")               # no weights
