"""The solver's history rules on the GPU: a diverging cycle stops with
MG_ERR_DIVERGED (weighted Jacobi with omega = 1.9 amplifies the highest
modes by |1 - 3.8| per sweep: the oracle's residual grows about 40x per
cycle), and the bf16-state refinement falls back to an FP32-stored iterate
when its steps stall -- forced here from the host by demanding a 1000x
reduction per step (MGX_BF16_STALL) -- and still converges."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_diverging_cycle_stops():
    import paper_1210_7774_amd as M
    n = 127
    say("divergence n=%d" % n)
    f = I.normal_rhs(n, 2, 50)
    s = M.Solver(n, 2, smoother="jacobi", omega=1.9, max_cycles=100)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    rc, st = s.solve(u, torch.from_numpy(f).cuda(), rtol=1e-10, raise_on_error=False)
    assert rc == M._abi.MG_ERR_DIVERGED
    h = np.array(st.history())
    say("  stopped after %d cycles, residual %.3e" % (st.cycles, h[-1]))
    assert 2 <= st.cycles < 100
    assert np.all(np.isfinite(h))
    ref = O.solve(f, opts=O.Opts(smoother=O.JACOBI, omega=1.9), tol=1e-10, maxc=st.cycles)
    assert np.allclose(h, ref.hist[: st.cycles + 1], rtol=1e-6)
    assert np.all(np.isfinite(u.cpu().numpy()))
    s.close()


@pytest.mark.parametrize("dim,n", [(2, 511), (3, 63)])
def test_bf16_state_falls_back_to_fp32(dim, n, monkeypatch):
    import paper_1210_7774_amd as M
    say("bf16 fallback d=%d n=%d" % (dim, n))
    f = I.normal_rhs(n, dim, 51)
    fd = torch.from_numpy(f).cuda()
    s = M.Solver(n, dim, precision="bf16")
    u = torch.zeros((n,) * dim, dtype=torch.float64, device="cuda")
    rc, st = s.solve(u, fd, rtol=1e-10)
    assert rc == 0 and st.fell_back == 0       # white noise: no stall
    monkeypatch.setenv("MGX_BF16_STALL", "0.001")
    u.zero_()
    rc, st = s.solve(u, fd, rtol=1e-10)
    say("  forced: status %d, %d steps, fell back %d" % (rc, st.cycles, st.fell_back))
    assert rc == M._abi.MG_FELL_BACK and st.fell_back == 1
    got = u.cpu().numpy()
    assert np.linalg.norm(O.residual(got, f)) / np.linalg.norm(f) <= 1e-10
    tight = O.solve(f, tol=1e-13)
    assert np.abs(got - tight.u).max() <= 1e-8 * np.abs(tight.u).max()
    monkeypatch.delenv("MGX_BF16_STALL")
    u.zero_()
    rc, st = s.solve(u, fd, rtol=1e-10)         # the next solve starts in bf16 again
    assert rc == 0 and st.fell_back == 0
    s.close()
