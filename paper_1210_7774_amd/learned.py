"""Learned smoother: training-pair generation from the plain solver's own
cycles, GPU training (forward, energy-norm loss, backward, Adam) and
inference.  Host orchestration only -- every pixel of work runs in the
library's kernels (include/mg.h, learned section); seeded random numbers
(initial weights, crop offsets, epoch orders) come from `inputs`.

Network (bias-free, zero padding): conv3x3 1->16, ReLU, 16->16, ReLU,
16->16, ReLU, 16->1; weights flat FP32, W[layer][co][ci][ky][kx].
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _abi, inputs
from ._abi import MGError

NWEIGHTS = _abi.NWEIGHTS


def _torch():
    import torch
    return torch


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _check(t, dtype, name, ndim=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s CUDA tensor" % (name, dtype))
    if ndim is not None and t.dim() != ndim:
        raise ValueError("%s must have %d dimensions" % (name, ndim))


def _err(rc, where):
    return MGError(rc, where, _abi.lib().mg_last_error(None).decode())


def scratch(batch: int, patch: int):
    """Device scratch for batches of `batch` maps of patch x patch."""
    nb = _abi.lib().mg_learned_scratch_bytes(int(batch), int(patch))
    if nb == 0:
        raise ValueError("bad batch / patch")
    return _torch().empty(nb, dtype=_torch().uint8, device="cuda")


def initial_weights(seed: int):
    """He-normal FP32 weights on the GPU."""
    return _torch().from_numpy(inputs.he_normal_weights(seed)).to("cuda")


def jacobi_weights(omega=0.8):
    """Weights for which N(s) = omega * s exactly (damped Jacobi on s):
    channel 0 carries relu(s), channel 1 relu(-s), the middle layers pass
    them through and the last returns omega * (ch0 - ch1).  FP32, on the GPU."""
    w = np.zeros(NWEIGHTS, dtype=np.float32)
    centre = 4                                  # tap (ky, kx) = (1, 1)
    w[0 * 9 + centre] = 1.0                     # layer 1: co 0 <- s
    w[1 * 9 + centre] = -1.0                    # layer 1: co 1 <- -s
    for base in (144, 144 + 2304):              # layers 2, 3: [co][ci][t]
        w[base + (0 * 16 + 0) * 9 + centre] = 1.0
        w[base + (1 * 16 + 1) * 9 + centre] = 1.0
    base = 144 + 2 * 2304                       # layer 4: [ci][t]
    w[base + 0 * 9 + centre] = omega
    w[base + 1 * 9 + centre] = -omega
    return _torch().from_numpy(w).to("cuda")


def jacobi_start(omega=0.8, noise_seed=7001, noise_scale=0.01):
    """Training start: the damped-Jacobi network plus small He-normal noise."""
    return (jacobi_weights(omega) + noise_scale * initial_weights(noise_seed)).contiguous()


def apply(s, w, work=None):
    """y = N(s) for s float32 [B, H, W] on the GPU."""
    _check(s, _torch().float32, "s", 3)
    _check(w, _torch().float32, "w")
    B, H, W = s.shape
    if work is None:
        work = scratch(B, max(H, W))
    y = _torch().empty_like(s)
    rc = _abi.lib().mg_learned_apply(_p(s), B, H, W, _p(w), _p(y), _p(work), work.numel(), _stream())
    if rc != _abi.MG_OK:
        raise _err(rc, "mg_learned_apply")
    return y


def loss_grad(s, e, a, w, border=5, work=None):
    """Energy-norm loss (float) and its gradient (FP32 CUDA tensor) over the
    B patches s, e, a (float32 [B, P, P])."""
    torch = _torch()
    for t, nm in ((s, "s"), (e, "e"), (a, "a")):
        _check(t, torch.float32, nm, 3)
    _check(w, torch.float32, "w")
    B, P, _ = s.shape
    if work is None:
        work = scratch(B, P)
    g = torch.empty(NWEIGHTS, dtype=torch.float32, device="cuda")
    loss = ctypes.c_double(0.0)
    rc = _abi.lib().mg_learned_loss_grad(_p(s), _p(e), _p(a), B, P, int(border), _p(w), ctypes.byref(loss), _p(g),
                                         _p(work), work.numel(), _stream())
    if rc != _abi.MG_OK:
        raise _err(rc, "mg_learned_loss_grad")
    return loss.value, g


@dataclass
class TrainResult:
    loss_hist: list
    steps: int
    ms: float


def train(S, E, A, w, epochs=30, batch=32, border=5, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, order_seed=7100,
          work=None) -> TrainResult:
    """Adam on the FP32 weights w (in place) over the pairs (S, E, A), float32
    [npairs, P, P] CUDA tensors; the pairs are visited in one seeded random
    order per epoch."""
    torch = _torch()
    for t, nm in ((S, "S"), (E, "E"), (A, "A")):
        _check(t, torch.float32, nm, 3)
    _check(w, torch.float32, "w")
    npairs, P, _ = S.shape
    order = torch.from_numpy(inputs.epoch_orders(npairs, epochs, order_seed)).to("cuda")
    if work is None:
        work = scratch(batch, P)
    o = _abi.TrainOptions(epochs, batch, P, border, lr, beta1, beta2, eps)
    hist = (ctypes.c_double * epochs)()
    st = _abi.TrainStats()
    rc = _abi.lib().mg_learned_train(_p(S), _p(E), _p(A), npairs, _p(order), ctypes.byref(o), _p(w), hist,
                                     ctypes.byref(st), _p(work), work.numel(), _stream())
    if rc != _abi.MG_OK:
        raise _err(rc, "mg_learned_train")
    return TrainResult(list(hist), st.steps, st.ms)


def crop(s, ustar, uk, a, offsets, patch, out=None):
    """Gather (s, e = ustar - uk, a) patches at the given (y0, x0) offsets
    (int32 [count, 2] CUDA tensor) of one n x n problem; float32 outputs."""
    torch = _torch()
    n = s.shape[0]
    for t, nm in ((s, "s"), (ustar, "ustar"), (uk, "uk")):
        _check(t, torch.float64, nm, 2)
    _check(a, torch.float64, "a", 2)
    _check(offsets, torch.int32, "offsets", 2)
    cnt = offsets.shape[0]
    y0 = offsets[:, 0].contiguous()
    x0 = offsets[:, 1].contiguous()
    if out is None:
        out = [torch.empty(cnt, patch, patch, dtype=torch.float32, device="cuda") for _ in range(3)]
    for t in out:
        _check(t, torch.float32, "out", 3)
        if tuple(t.shape) != (cnt, patch, patch):
            raise ValueError("out tensors must be [count, patch, patch]")
    rc = _abi.lib().mg_learned_crop(_p(s), _p(ustar), _p(uk), _p(a), n, _p(y0), _p(x0), cnt, patch, _p(out[0]),
                                    _p(out[1]), _p(out[2]), _stream())
    if rc != _abi.MG_OK:
        raise _err(rc, "mg_learned_crop")
    return out


def make_pairs(problems, cycles=10, crops=100, patch=64, seed=7200, solve_rtol=1e-12, stages=("pre", "post")):
    """Training pairs from the plain FP64 red-black Gauss-Seidel solver's own
    cycles, taken where the cycle applies its smoother: for each problem
    (a nodal [(n+2)^2], f [n^2], numpy FP64) the reference solution u*
    (solved to solve_rtol); then for each of `cycles` V(2,2) cycles from
    u = 0, the state the pre-smoother sees (u_k, the cycle's start) and the
    state the post-smoother sees (u_k after 2 pre-sweeps and the coarse-grid
    correction, from a V(2,0) cycle) each give s = D^-1 (f - A u) and
    e = u* - u, cropped at `crops` seeded offsets.  Stage "noise" adds pairs
    of a seeded white-noise error e with s = D^-1 A e (all error modes, the
    smoothing property).  Returns float32 CUDA tensors S, E, A of
    [count, patch, patch]."""
    from . import Solver
    torch = _torch()
    stages = tuple(stages)
    for st in stages:
        if st not in ("pre", "post", "noise"):
            raise ValueError("stages are 'pre', 'post' and 'noise'")
    total = len(problems) * cycles * crops * len(stages)
    S = torch.empty(total, patch, patch, dtype=torch.float32, device="cuda")
    E = torch.empty_like(S)
    A = torch.empty_like(S)
    q = 0
    for pi, (a_np, f_np) in enumerate(problems):
        n = f_np.shape[0]
        a = torch.from_numpy(np.ascontiguousarray(a_np)).to("cuda")
        f = torch.from_numpy(np.ascontiguousarray(f_np)).to("cuda")
        sol = Solver(n, 2, a=a, max_cycles=200)
        pre_only = Solver(n, 2, a=a, nu1=2, nu2=0) if "post" in stages else None
        ustar = torch.zeros_like(f)
        rc, st = sol.solve(ustar, f, rtol=solve_rtol, raise_on_error=True)
        if st.rel_res > 10 * solve_rtol:
            raise RuntimeError("reference solve reached only %.3g" % st.rel_res)
        u = torch.zeros_like(f)
        zero = torch.zeros_like(f)
        w = torch.empty_like(f)
        s = torch.empty_like(f)
        for k in range(cycles):
            for si, stage in enumerate(stages):
                if stage == "noise":
                    # white-noise error e: s = D^-1 A e is the scaled
                    # residual of u = -e for f = 0, and e = 0 - u
                    w.copy_(torch.from_numpy(-inputs.normal_rhs(n, 2, seed + 500000 + 1000 * pi + k)))
                    sol.scaled_residual(w, zero, s)
                    crop(s, zero, w, a, torch.from_numpy(
                        inputs.crop_offsets(n, patch, crops, seed + 1000 * pi + 10 * k + si)).to("cuda"), patch,
                        out=(S[q:q + crops], E[q:q + crops], A[q:q + crops]))
                    q += crops
                    continue
                if stage == "pre":
                    src = u
                else:
                    w.copy_(u)
                    pre_only.vcycle(w, f)
                    src = w
                sol.scaled_residual(src, f, s)
                off = torch.from_numpy(inputs.crop_offsets(n, patch, crops, seed + 1000 * pi + 10 * k + si)).to("cuda")
                crop(s, ustar, src, a, off, patch, out=(S[q:q + crops], E[q:q + crops], A[q:q + crops]))
                q += crops
            sol.vcycle(u, f)
        sol.close()
        if pre_only is not None:
            pre_only.close()
    return S, E, A
