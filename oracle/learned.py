"""Oracle for the learned smoother: a plain numpy FP64 reference of the
network, its energy-norm loss, the hand-written backward pass and Adam.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Conventions:
  * network N: 3x3 convolutions 1 -> 16 -> 16 -> 16 -> 1, ReLU after the
    first three, no biases, zero padding; output pixel (i, j) of a layer uses
    input pixel (i + ky - 1, j + kx - 1) with weight W[co, ci, ky, kx];
  * flat weight vector: the four layers' W arrays in order, each C-ordered
    (144 + 2304 + 2304 + 144 = 4896 numbers);
  * patches are [B, P, P] arrays indexed [b, i (y), j (x)];
  * the smoother step is s = D^-1 (f - A u), u <- u + N(s);
  * energy of w on the window V (the patch minus a border of `border` pixels):
    E_V(w) = sum over faces with both ends in V of a_f (w_1 - w_2)^2, a_f the
    harmonic mean of the nodal coefficient at the face's ends (the 1/h^2 of the
    operator cancels in the loss ratio);
  * loss L = mean_b E_V(e_b - N(s_b)) / E_V(e_b).
Optionally every layer input, the weights and the stored activations are
rounded to bfloat16 (round to nearest even), as the GPU stores them.
"""
from __future__ import annotations

import numpy as np

SHAPES = [(16, 1), (16, 16), (16, 16), (1, 16)]   # (c_out, c_in) per layer
NWEIGHTS = sum(co * ci * 9 for co, ci in SHAPES)   # 4896


def bf16(x):
    """Round float64 values to the nearest bfloat16 (via float32, ties to even),
    returned as float64."""
    x32 = np.asarray(x, dtype=np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    nan = np.isnan(x32)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    out = b.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def unflatten(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == NWEIGHTS
    out, k = [], 0
    for co, ci in SHAPES:
        m = co * ci * 9
        out.append(w[k:k + m].reshape(co, ci, 3, 3))
        k += m
    return out


def flatten(ws):
    return np.concatenate([w.reshape(-1) for w in ws])


def conv3x3(x, w):
    """y[b, co, i, j] = sum_{ci, ky, kx} w[co, ci, ky, kx] x[b, ci, i+ky-1, j+kx-1]
    with zero padding; x [B, Ci, H, W], w [Co, Ci, 3, 3]."""
    B, Ci, H, W = x.shape
    xp = np.zeros((B, Ci, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((B, w.shape[0], H, W))
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("oc,bchw->bohw", w[:, :, ky, kx], xp[:, :, ky:ky + H, kx:kx + W])
    return y


def conv3x3_dgrad(dy, w):
    """dx[b, ci, i, j] = sum_{co, ky, kx} w[co, ci, ky, kx] dy[b, co, i-ky+1, j-kx+1]."""
    B, Co, H, W = dy.shape
    dyp = np.zeros((B, Co, H + 2, W + 2))
    dyp[:, :, 1:-1, 1:-1] = dy
    dx = np.zeros((B, w.shape[1], H, W))
    for ky in range(3):
        for kx in range(3):
            # dy at (i - ky + 1, j - kx + 1) sits at padded (i - ky + 2, j - kx + 2)
            dx += np.einsum("oc,bohw->bchw", w[:, :, ky, kx], dyp[:, :, 2 - ky:2 - ky + H, 2 - kx:2 - kx + W])
    return dx


def conv3x3_wgrad(x, dy):
    """dw[co, ci, ky, kx] = sum_{b, i, j} dy[b, co, i, j] x[b, ci, i+ky-1, j+kx-1]."""
    B, Ci, H, W = x.shape
    xp = np.zeros((B, Ci, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dw = np.zeros((dy.shape[1], Ci, 3, 3))
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.einsum("bohw,bchw->oc", dy, xp[:, :, ky:ky + H, kx:kx + W])
    return dw


def forward(s, w, bf16_emul=False, keep=False):
    """N(s) for s [B, P, P]; returns y [B, P, P] (and the activations)."""
    ws = unflatten(w)
    if bf16_emul:
        ws = [bf16(x) for x in ws]
    x = np.asarray(s, dtype=np.float64)[:, None]
    if bf16_emul:
        x = bf16(x)
    acts = [x]
    for li, wl in enumerate(ws):
        z = conv3x3(x, wl)
        if li < 3:
            x = np.maximum(z, 0.0)
            if bf16_emul:
                x = bf16(x)
            acts.append(x)
        else:
            x = z
    y = x[:, 0]
    return (y, acts, ws) if keep else y


def face_weights(a):
    """Harmonic face means of a nodal patch a [B, P, P]: (horizontal faces
    [B, P, P-1] between (i, j) and (i, j+1); vertical faces [B, P-1, P])."""
    ax = 2 * a[:, :, :-1] * a[:, :, 1:] / (a[:, :, :-1] + a[:, :, 1:])
    ay = 2 * a[:, :-1, :] * a[:, 1:, :] / (a[:, :-1, :] + a[:, 1:, :])
    return ax, ay


def window_masks(P, border):
    inside = np.zeros(P, dtype=bool)
    inside[border:P - border] = True
    mx = inside[None, :-1] & inside[None, 1:] & inside[:, None]      # horizontal faces [P, P-1]
    my = inside[:-1, None] & inside[1:, None] & inside[None, :]      # vertical faces [P-1, P]
    return mx, my


def energy(w, a, border=5):
    """E_V(w) per patch, [B]."""
    ax, ay = face_weights(a)
    mx, my = window_masks(w.shape[-1], border)
    dx = w[:, :, 1:] - w[:, :, :-1]
    dy = w[:, 1:, :] - w[:, :-1, :]
    return (ax * dx * dx * mx).sum(axis=(1, 2)) + (ay * dy * dy * my).sum(axis=(1, 2))


def energy_operator(w, a, border=5):
    """(A_V w)_p = sum over window faces f at p of a_f (w_p - w_other) = (1/2) dE_V/dw."""
    ax, ay = face_weights(a)
    mx, my = window_masks(w.shape[-1], border)
    gx = ax * (w[:, :, 1:] - w[:, :, :-1]) * mx
    gy = ay * (w[:, 1:, :] - w[:, :-1, :]) * my
    out = np.zeros_like(w)
    out[:, :, 1:] += gx
    out[:, :, :-1] -= gx
    out[:, 1:, :] += gy
    out[:, :-1, :] -= gy
    return out


def loss(s, e, a, w, border=5, bf16_emul=False):
    y = forward(s, w, bf16_emul)
    return float(np.mean(energy(e - y, a, border) / energy(e, a, border)))


def loss_and_grad(s, e, a, w, border=5, bf16_emul=False):
    """L and dL/dw (flat) by the hand-written backward pass."""
    B = s.shape[0]
    y, acts, ws = forward(s, w, bf16_emul, keep=True)
    E0 = energy(e, a, border)
    resid = e - y
    L = float(np.mean(energy(resid, a, border) / E0))
    # dL/dy = -(2/B) A_V(e - y) / E(e)
    dy = (-2.0 / B) * energy_operator(resid, a, border) / E0[:, None, None]
    g = dy[:, None]
    grads = [None] * 4
    for li in range(3, -1, -1):
        x = acts[li]
        grads[li] = conv3x3_wgrad(x, g)
        if li > 0:
            g = conv3x3_dgrad(g, ws[li]) * (acts[li] > 0)
    return L, flatten(grads)


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t = 1, 2, ...); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def he_normal(rng):
    """He-normal initial weights (std sqrt(2 / fan_in), fan_in = 9 c_in) drawn
    from the given numpy Generator, flat."""
    return flatten([rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (9 * ci)) for co, ci in SHAPES])


def omega_identity(omega):
    """Weights for which N(s) = omega * s exactly: channel 0 carries relu(s),
    channel 1 relu(-s), layers 2 and 3 pass them through, layer 4 returns
    omega (ch0 - ch1)."""
    ws = [np.zeros((co, ci, 3, 3)) for co, ci in SHAPES]
    ws[0][0, 0, 1, 1] = 1.0
    ws[0][1, 0, 1, 1] = -1.0
    for li in (1, 2):
        ws[li][0, 0, 1, 1] = 1.0
        ws[li][1, 1, 1, 1] = 1.0
    ws[3][0, 0, 1, 1] = omega
    ws[3][0, 1, 1, 1] = -omega
    return flatten(ws)


def scaled_residual(u, f, a, h):
    """s = D^-1 (f - A u) on a full 2D grid (interior [n, n], nodal a
    [n+2, n+2]) in FP64, using the C oracle's residual."""
    import oracle as O
    r = O.residual(np.ascontiguousarray(u), np.ascontiguousarray(f), a=np.ascontiguousarray(a), h=h)
    n = u.shape[0]
    c = a[1:-1, 1:-1]
    hm = lambda p, q: 2 * p * q / (p + q)  # noqa: E731
    D = (hm(c, a[1:-1, :-2]) + hm(c, a[1:-1, 2:]) + hm(c, a[:-2, 1:-1]) + hm(c, a[2:, 1:-1])) / (h * h)
    assert D.shape == (n, n)
    return r / D


def learned_step(u, f, a, w, h, bf16_emul=False):
    """u + N(D^-1 (f - A u)) on the full grid (the network sees the whole
    interior; zero padding is the Dirichlet boundary)."""
    s = scaled_residual(u, f, a, h)
    return u + forward(s[None], w, bf16_emul)[0]


def learned_vcycle(u, f, a, w, nu1=2, nu2=2, bf16_emul=False):
    """V-cycle whose finest-level sweeps are learned steps; coarser levels are
    the plain red-black Gauss-Seidel V-cycle of the C oracle."""
    import oracle as O
    n = u.shape[0]
    h = 1.0 / (n + 1)
    for _ in range(nu1):
        u = learned_step(u, f, a, w, h, bf16_emul)
    r = O.residual(u, f, a=a)
    fc = O.restrict(r)
    ac = O.coarsen_coef(a, 2)
    uc = np.zeros_like(fc)
    O.vcycle(uc, fc, a=ac, h=2 * h)
    u = O.prolong_add(uc, u.copy())
    for _ in range(nu2):
        u = learned_step(u, f, a, w, h, bf16_emul)
    return u
