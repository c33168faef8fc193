"""Pins of the learned-smoother oracle (oracle/learned.py) against torch's own
CPU convolution, autograd and Adam (independent library routines), finite
differences, and the network's exact special cases."""
import numpy as np
import pytest
import torch

import oracle as O
import oracle.learned as LN
from paper_1210_7774_amd import inputs as I


def rand_patches(B=2, P=16, seed=0):
    rng = np.random.default_rng(seed)
    s = rng.standard_normal((B, P, P))
    e = rng.standard_normal((B, P, P))
    a = np.exp(rng.standard_normal((B, P, P)) * 0.5)
    return s, e, a


def test_weight_count():
    assert LN.NWEIGHTS == 4896


def test_conv_matches_torch():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 16, 9, 11))
    w = rng.standard_normal((16, 16, 3, 3))
    want = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(w), padding=1).numpy()
    assert np.abs(LN.conv3x3(x, w) - want).max() <= 1e-12


def test_dgrad_wgrad_match_torch_autograd():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 16, 8, 7))
    w = rng.standard_normal((16, 16, 3, 3))
    dy = rng.standard_normal((2, 16, 8, 7))
    xt = torch.from_numpy(x).requires_grad_(True)
    wt = torch.from_numpy(w).requires_grad_(True)
    y = torch.nn.functional.conv2d(xt, wt, padding=1)
    y.backward(torch.from_numpy(dy))
    assert np.abs(LN.conv3x3_dgrad(dy, w) - xt.grad.numpy()).max() <= 1e-11
    assert np.abs(LN.conv3x3_wgrad(x, dy) - wt.grad.numpy()).max() <= 1e-11


def test_q13_gradient_finite_differences():
    s, e, a = rand_patches(2, 16, 3)
    w = LN.he_normal(np.random.default_rng(7000))
    L, g = LN.loss_and_grad(s, e, a, w, border=3)
    rng = np.random.default_rng(4)
    idx = rng.choice(LN.NWEIGHTS, 20, replace=False)
    for k in idx:
        hstep = 1e-6 * max(1.0, abs(w[k]))
        wp, wm = w.copy(), w.copy()
        wp[k] += hstep
        wm[k] -= hstep
        fd = (LN.loss(s, e, a, wp, border=3) - LN.loss(s, e, a, wm, border=3)) / (2 * hstep)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (k, fd, g[k])


def test_gradient_matches_torch_autograd():
    """The whole hand-written backward pass against torch autograd of the
    same forward and loss written in torch (CPU, float64)."""
    s, e, a = rand_patches(3, 14, 5)
    w = LN.he_normal(np.random.default_rng(11))
    L, g = LN.loss_and_grad(s, e, a, w, border=2)
    ws = [torch.from_numpy(x.copy()).requires_grad_(True) for x in LN.unflatten(w)]
    x = torch.from_numpy(s)[:, None]
    for li, wl in enumerate(ws):
        x = torch.nn.functional.conv2d(x, wl, padding=1)
        if li < 3:
            x = torch.relu(x)
    y = x[:, 0]
    at = torch.from_numpy(a)
    ax = 2 * at[:, :, :-1] * at[:, :, 1:] / (at[:, :, :-1] + at[:, :, 1:])
    ay = 2 * at[:, :-1, :] * at[:, 1:, :] / (at[:, :-1, :] + at[:, 1:, :])
    mx, my = LN.window_masks(14, 2)
    mx, my = torch.from_numpy(mx), torch.from_numpy(my)

    def E(v):
        return ((ax * (v[:, :, 1:] - v[:, :, :-1]) ** 2 * mx).sum((1, 2))
                + (ay * (v[:, 1:, :] - v[:, :-1, :]) ** 2 * my).sum((1, 2)))

    et = torch.from_numpy(e)
    Lt = (E(et - y) / E(et)).mean()
    Lt.backward()
    gt = np.concatenate([wl.grad.numpy().reshape(-1) for wl in ws])
    assert abs(L - Lt.item()) <= 1e-12
    assert np.abs(g - gt).max() <= 1e-10 * max(1.0, np.abs(gt).max())


def test_energy_is_quadratic_form():
    s, e, a = rand_patches(1, 10, 6)
    E = LN.energy(e, a, border=2)[0]
    Ae = LN.energy_operator(e, a, border=2)
    assert abs(E - float((e * Ae).sum())) <= 1e-12 * E


def test_q14_special_cases():
    s, e, a = rand_patches(2, 12, 7)
    assert np.all(LN.forward(s, np.zeros(LN.NWEIGHTS)) == 0.0)
    for om in (0.5, 0.75):
        y = LN.forward(s, LN.omega_identity(om))
        assert np.abs(y - om * s).max() <= 1e-15 * np.abs(s).max()
        yb = LN.forward(s, LN.omega_identity(om), bf16_emul=True)
        assert np.array_equal(yb, om * LN.bf16(s))


def test_q14_identity_network_is_jacobi():
    n = 31
    a = I.lognormal_coef_2d(n, 4020)
    f = I.normal_rhs(n, 2, 4520)
    u = I.normal_rhs(n, 2, 4521) * 1e-3
    h = 1.0 / (n + 1)
    got = LN.learned_step(u, f, a, LN.omega_identity(0.5), h)
    want = O.sweep(u.copy(), f, a=a, kind=O.JACOBI, omega=0.5)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_positive_homogeneity():
    s, e, a = rand_patches(2, 12, 8)
    w = LN.he_normal(np.random.default_rng(9))
    y1 = LN.forward(s, w)
    y2 = LN.forward(8.0 * s, w)
    assert np.array_equal(8.0 * y1, y2)
    yb1 = LN.forward(s, w, bf16_emul=True)
    yb2 = LN.forward(8.0 * s, w, bf16_emul=True)
    assert np.array_equal(8.0 * yb1, yb2)


def test_adam_matches_torch():
    rng = np.random.default_rng(10)
    w = rng.standard_normal(50)
    wt = torch.from_numpy(w.copy()).requires_grad_(True)
    opt = torch.optim.Adam([wt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for t in range(1, 6):
        g = rng.standard_normal(50)
        w, m, v = LN.adam_step(w, g, m, v, t)
        opt.zero_grad()
        wt.grad = torch.from_numpy(g)
        opt.step()
    assert np.abs(w - wt.detach().numpy()).max() <= 1e-12


def test_bf16_helper_matches_torch():
    x = np.random.default_rng(12).standard_normal(5000) * 100
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(LN.bf16(x), want)


@pytest.mark.slow
def test_learned_vcycle_with_jacobi_weights_converges():
    n = 63
    a = I.lognormal_coef_2d(n, 4030)
    f = I.normal_rhs(n, 2, 4530)
    u = np.zeros_like(f)
    hist = [1.0]
    for _ in range(8):
        u = LN.learned_vcycle(u, f, a, LN.omega_identity(0.8))
        hist.append(np.linalg.norm(O.residual(u, f, a=a)) / np.linalg.norm(f))
    assert hist[-1] < 1e-3 and all(b < c for b, c in zip(hist[1:], hist[:-1]))
