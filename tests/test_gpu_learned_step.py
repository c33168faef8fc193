"""The solver's fused learned step (one kernel: scaled residual, the four
convolution layers on MFMA, the update) element by element against the
oracle's network (oracle/learned.py, FP64 with the GPU's bf16 rounding points
emulated), through mg_learned_step, and one learned V-cycle of the solver
against the oracle's learned V-cycle.  Both forms of the kernel are covered:
the row-marching one (the default; strips of 56 columns, R rows per
workgroup, including R that leave a ragged last run) and the tiled one
(MGX_LSTEP_TILED=1).

Tolerances: the GPU accumulates each layer in FP32 in its own order and
computes s in FP32 with hardware reciprocals, so a bf16 rounding of s or of an
activation can land one bf16 ulp (2^-8 relative) away from the oracle's where
the value sits near a rounding boundary; those flips are rare and local.  With
inputs whose s is exact in bf16 (a = 1, e = 0, f a bf16 multiple of 4/h^2) the
update agrees to relative L2 2e-3; with log-normal coefficients and random
iterates to 1e-2, and every value to 3e-2 of the largest update.  A wrong tap,
channel, layer or sign moves the update by O(1) and fails both.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle.learned as LN
from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, params=["march", "tiled"])
def step_form(request, monkeypatch):
    """Every test runs on both forms of the fused step (the library reads the
    switch at each launch)."""
    monkeypatch.setenv("MGX_LSTEP_TILED", "1" if request.param == "tiled" else "0")
    return request.param


def say(*a):
    print(*a, flush=True)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def bf(x):
    return torch.from_numpy(np.asarray(x, dtype=np.float64)).to(torch.float32).to(torch.bfloat16).to(
        torch.float32).numpy().astype(np.float64)


def rel_l2(got, want):
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def gpu_step(e, f, a, w, prec):
    """mg_learned_step on host float64 data (already representable in the
    state / float types); returns e_out as float64."""
    from paper_1210_7774_amd import _abi
    L = _abi.lib()
    n = e.shape[0]
    if prec == "f32":
        et = torch.from_numpy(e.astype(np.float32)).cuda()
    else:
        et = torch.from_numpy(e.astype(np.float32)).to(torch.bfloat16).cuda()
    eo = torch.empty_like(et)
    ft = torch.from_numpy(f.astype(np.float32)).cuda()
    at = torch.from_numpy(a.astype(np.float32)).cuda()
    wt = torch.from_numpy(np.asarray(w, dtype=np.float32)).cuda()
    nb = L.mg_learned_scratch_bytes(1, 3)
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    pr = _abi.MG_P_F32_IR if prec == "f32" else _abi.MG_P_F32_BF16_IR
    rc = L.mg_learned_step(_p(et), _p(eo), _p(ft), _p(at), n, pr, _p(wt), _p(scratch), nb, stream)
    assert rc == _abi.MG_OK, L.mg_last_error(None)
    return eo.to(torch.float32).cpu().numpy().astype(np.float64)


def he_net(seed):
    return I.he_normal_weights(seed).astype(np.float64)


@pytest.mark.parametrize("n,prec", [(255, "f32"), (255, "bf16"), (1023, "f32"), (1023, "bf16"), (77, "f32"),
                                    (7, "f32"), (17, "bf16")])
def test_fused_step_matches_oracle(n, prec):
    """Random He-normal network (every tap and channel of every layer in
    use), log-normal coefficients, a random iterate: n = 255 / 1023 span
    many 64 x 8 tiles or 56-column strips with ragged edges; 77 is not a
    multiple of any of them; 7 and 17 are narrower than one tile, strip or
    16-column MFMA segment (every job masked)."""
    say("fused learned step n=%d %s" % (n, prec))
    h = 1.0 / (n + 1)
    a = f32(I.lognormal_coef_2d(n, 4060 + n))
    f = f32(I.normal_rhs(n, 2, 4560 + n))
    e = 0.25 * h * h * I.normal_rhs(n, 2, 4660 + n)
    e = f32(e) if prec == "f32" else bf(e)
    w = f32(he_net(70 + n))
    got = gpu_step(e, f, a, w, prec)
    want = LN.learned_step(e, f, a, w, h, bf16_emul=True)
    dg, dw = got - e, want - e
    r = rel_l2(dg, dw)
    m = float(np.abs(dg - dw).max() / np.abs(dw).max())
    say("  rel L2 %.3e, max %.3e of the largest update" % (r, m))
    assert r <= 1e-2
    assert m <= 3e-2


@pytest.mark.parametrize("rows", [4, 13, 40, 300])
def test_march_rows_per_workgroup(rows, step_form, monkeypatch):
    """The row-marching form with R rows per workgroup: 4 (shorter than the
    pipeline fill), 13 (a ragged last run of 8 rows at n = 255), 40 and 300
    (one run per strip)."""
    if step_form != "march":
        pytest.skip("rows per workgroup belong to the row-marching form")
    monkeypatch.setenv("MGX_LSTEP_ROWS", str(rows))
    n = 255
    say("fused learned step n=%d, %d rows per workgroup" % (n, rows))
    h = 1.0 / (n + 1)
    a = f32(I.lognormal_coef_2d(n, 4061))
    f = f32(I.normal_rhs(n, 2, 4561))
    e = f32(0.25 * h * h * I.normal_rhs(n, 2, 4661))
    w = f32(he_net(72))
    got = gpu_step(e, f, a, w, "f32")
    want = LN.learned_step(e, f, a, w, h, bf16_emul=True)
    dg, dw = got - e, want - e
    r = rel_l2(dg, dw)
    m = float(np.abs(dg - dw).max() / np.abs(dw).max())
    say("  rel L2 %.3e, max %.3e of the largest update" % (r, m))
    assert r <= 1e-2
    assert m <= 3e-2


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_fused_step_exact_inputs(prec):
    """a = 1 and e = 0 make s = h^2 f / 4 exact: with f = bf16 values times
    4 / h^2 (a power of two) the network's input is exactly the oracle's."""
    n = 255
    say("fused learned step, exact inputs", prec)
    h = 1.0 / (n + 1)
    a = np.ones((n + 2, n + 2))
    f = bf(I.normal_rhs(n, 2, 4700)) * (4.0 / (h * h))
    e = np.zeros((n, n))
    w = f32(he_net(71))
    got = gpu_step(e, f, a, w, prec)
    want = LN.learned_step(e, f, a, w, h, bf16_emul=True)
    if prec == "bf16":
        want = bf(want)
    r = rel_l2(got, want)
    say("  rel L2 %.3e" % r)
    assert r <= 2e-3
    # the zero network gives e back exactly, the omega-identity one omega bf16(s)
    z = gpu_step(e, f, a, np.zeros(LN.NWEIGHTS), prec)
    assert np.array_equal(z, e)
    om = gpu_step(e, f, a, LN.omega_identity(0.5), prec)
    assert np.array_equal(om, 0.5 * bf(h * h * f / 4.0))


def test_learned_vcycle_matches_oracle():
    """One refinement step of the learned-smoother solver (FP32 inner cycle,
    learned finest-level steps, red-black Gauss-Seidel below) against the
    oracle's learned V-cycle on the FP32 inner problem."""
    import paper_1210_7774_amd as M
    n = 255
    say("learned V-cycle vs oracle n=%d" % n)
    a64 = I.lognormal_coef_2d(n, 4061)
    f64 = I.normal_rhs(n, 2, 4561)
    w = f32(LN.omega_identity(0.5) + 0.1 * he_net(72))
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    s = M.Solver(n, 2, a=torch.from_numpy(a64).cuda(), precision="f32", smoother="learned", learned=wt)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    s.vcycle(u, torch.from_numpy(f64).cuda())
    got = u.cpu().numpy()
    want = LN.learned_vcycle(np.zeros((n, n)), f32(f64), f32(a64), w, bf16_emul=True)
    r = rel_l2(got, want)
    say("  rel L2 %.3e" % r)
    assert r <= 2e-2
    s.close()
