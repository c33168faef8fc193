"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds input generation only -- no operator, smoother or transfer
arithmetic -- so both the HIP path and the oracle may take their data from it.
Every generator uses numpy ``Generator(PCG64(seed))``; arrays are float64,
interior-only, x fastest (shape ``(n,)*d``), coefficients on the ``(n+2)^d``
nodes including the boundary.
"""
from __future__ import annotations

import math

import numpy as np

C4_SIZES = (127, 255, 511, 1023)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def grid_x(n: int) -> np.ndarray:
    """Interior node coordinates x_i = i h, i = 1..n, h = 1/(n+1)."""
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def sine_plus_noise_1d(n: int = 1023, seed: int = 1, amp: float = 1e-3) -> np.ndarray:
    """1D rhs: pi^2 sin(pi x_i) (= -u'' for u = sin(pi x)) plus i.i.d.
    uniform noise on [-amp, amp]."""
    x = grid_x(n)
    return math.pi ** 2 * np.sin(math.pi * x) + rng(seed).uniform(-amp, amp, size=n)


def normal_rhs(n: int, d: int, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) right-hand side on the n^d interior nodes."""
    return rng(seed).standard_normal((n,) * d)


def uniform_field(shape, seed: int) -> np.ndarray:
    return rng(seed).uniform(0.0, 1.0, size=shape)


def gaussian_field_2d(n: int, seed: int, sigma: float = 1.0, ell: float = 1.0 / 16) -> np.ndarray:
    """Stationary Gaussian random field on the (n+2)^2 nodes of [0,1]^2
    (boundary included), squared-exponential covariance
    sigma^2 exp(-r^2 / (2 ell^2)), by circulant embedding on an M x M periodic
    grid of the same spacing, M the next power of two >= (n+2) + ceil(6 ell/h).
    Negative embedding eigenvalues are clipped to 0."""
    h = 1.0 / (n + 1)
    need = (n + 2) + int(math.ceil(6.0 * ell / h))
    M = 1 << (need - 1).bit_length()
    k = np.arange(M)
    dist = np.minimum(k, M - k) * h
    r2 = dist[:, None] ** 2 + dist[None, :] ** 2
    c = sigma ** 2 * np.exp(-r2 / (2.0 * ell ** 2))
    lam = np.fft.fft2(c).real
    lam = np.maximum(lam, 0.0)
    xi = rng(seed).standard_normal((M, M))
    g = np.fft.ifft2(np.sqrt(lam) * np.fft.fft2(xi)).real
    return np.ascontiguousarray(g[: n + 2, : n + 2])


def lognormal_coef_2d(n: int, seed: int, sigma: float = 1.0, ell: float = 1.0 / 16) -> np.ndarray:
    """Nodal diffusion coefficient a = exp(g), g the field above."""
    return np.exp(gaussian_field_2d(n, seed, sigma, ell))


def batch_sizes(count: int = 256, seed: int = 40, sizes=C4_SIZES) -> np.ndarray:
    """Grid sizes of an uneven batch: n drawn uniformly from ``sizes``."""
    return rng(seed).choice(np.asarray(sizes), size=count)


def batch_problem(count: int = 256, sizes_seed: int = 40, coef_seed0: int = 4000, rhs_seed0: int = 4500,
                  sizes=C4_SIZES):
    """The uneven batch of 2D variable-coefficient systems: for system s,
    n_s from ``batch_sizes``, a = exp(g) with g seeded coef_seed0 + s,
    f ~ N(0,1) seeded rhs_seed0 + s."""
    ns = batch_sizes(count, sizes_seed, sizes)
    out = []
    for s, n in enumerate(ns):
        n = int(n)
        out.append((n, lognormal_coef_2d(n, coef_seed0 + s), normal_rhs(n, 2, rhs_seed0 + s)))
    return out


# ---- learned smoother: seeded draws (the method's random numbers, passed in) --
LEARNED_SHAPES = [(16, 1), (16, 16), (16, 16), (1, 16)]   # (c_out, c_in) per layer


def he_normal_weights(seed: int) -> np.ndarray:
    """He-normal initial weights, flat FP32 in the layer order
    W[layer][co][ci][ky][kx]: N(0, 2 / (9 c_in)) per layer."""
    g = rng(seed)
    parts = [g.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (9 * ci)) for co, ci in LEARNED_SHAPES]
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def crop_offsets(n: int, patch: int, count: int, seed: int) -> np.ndarray:
    """count (y0, x0) offsets of patch x patch crops inside an n x n interior,
    uniform over the valid range; int32 [count, 2]."""
    return rng(seed).integers(0, n - patch + 1, size=(count, 2)).astype(np.int32)


def epoch_orders(npairs: int, epochs: int, seed: int) -> np.ndarray:
    """One random permutation of the pairs per epoch, int32 [epochs * npairs]."""
    g = rng(seed)
    return np.concatenate([g.permutation(npairs) for _ in range(epochs)]).astype(np.int32)


# ---- vector bytecode: seeded random programs (instruction lists as data) ------
# A view is (base, offset, shape, strides) in elements; an instruction is
# (op, out_view, inputs) with inputs views or float constants.  Op names are
# plain strings; no operation is evaluated here.
VEC_ELEMENTWISE = ("copy", "add", "subtract", "multiply", "divide", "maximum", "minimum", "negative", "absolute",
                   "sqrt", "greater", "less_equal", "where")
VEC_MATH = ("exp", "log", "sin", "cos", "tanh", "power")
VEC_ARITY = {"copy": 1, "negative": 1, "absolute": 1, "sqrt": 1, "exp": 1, "log": 1, "sin": 1, "cos": 1, "tanh": 1,
             "add": 2, "subtract": 2, "multiply": 2, "divide": 2, "maximum": 2, "minimum": 2, "power": 2,
             "greater": 2, "greater_equal": 2, "less": 2, "less_equal": 2, "equal": 2, "not_equal": 2,
             "where": 3, "add_reduce": 1, "maximum_reduce": 1}


def vector_program(seed: int, ninstr: int = 16, nbases: int = 4, rows: int = 6, cols: int = 9, ops=VEC_ELEMENTWISE,
                   reductions: bool = False):
    """A random batch over `nbases` 2D bases of (rows + 4) x (2 cols + 4)
    elements (row-major) plus one temporary base per instruction, every
    instruction on a rows x cols index space.  Views are windows of a base:
    identical to earlier ones, shifted by one row or column, interleaved
    (every other column), reversed, or the transposed-stride form of a square
    window, so that the blockable rule both fuses and splits.  Returns
    (bases, instrs, data): bases = [(nelem, dtype)], data = the initial base
    contents (U(0.5, 1.5); temporaries start as zeros)."""
    g = rng(seed)
    R, C = rows, cols
    W = 2 * cols + 4
    nel = (rows + 4) * W
    bases = [(nel, "f64") for _ in range(nbases)]
    data = [g.uniform(0.5, 1.5, size=nel) for _ in range(nbases)]

    def window(b):
        kind = g.integers(0, 6)
        r0, c0 = int(g.integers(0, 3)), int(g.integers(0, 3))
        if kind == 3 and cols >= 2:      # every other column (C elements from 2C - 1 columns)
            c0 = int(g.integers(0, 2))
            if c0 + 2 * (C - 1) >= W:
                kind = 0
            else:
                return (b, r0 * W + c0, (R, C), (W, 2))
        if kind == 4:                    # reversed rows
            return (b, (r0 + R - 1) * W + c0, (R, C), (-W, 1))
        return (b, r0 * W + c0, (R, C), (W, 1))

    views = []
    instrs = []
    for i in range(ninstr):
        red = reductions and g.random() < 0.15
        op = ("add_reduce" if g.random() < 0.5 else "maximum_reduce") if red else ops[int(g.integers(0, len(ops)))]
        ins = []
        for _ in range(VEC_ARITY[op]):
            u = g.random()
            if u < 0.15 and op not in ("add_reduce", "maximum_reduce"):
                ins.append(float(np.round(g.uniform(0.25, 2.0), 3)))
            elif u < 0.55 and views:
                ins.append(views[int(g.integers(0, len(views)))])
            else:
                v = window(int(g.integers(0, nbases)))
                views.append(v)
                ins.append(v)
        if all(not isinstance(x, tuple) for x in ins):
            v = window(int(g.integers(0, nbases)))
            ins[0] = v
        if red:
            bases.append((1, "f64"))
            data.append(np.zeros(1))
            out = (len(bases) - 1, 0, (1,), (1,))
        else:
            u = g.random()
            if u < 0.3:
                bases.append((R * C, "f64"))   # a fresh temporary
                data.append(np.zeros(R * C))
                out = (len(bases) - 1, 0, (R, C), (C, 1))
            elif u < 0.65 and views:
                out = views[int(g.integers(0, len(views)))]
            else:
                out = window(int(g.integers(0, nbases)))
            if out[3][1] == 0:
                out = window(int(g.integers(0, nbases)))
            views.append(out)
        instrs.append((op, out, tuple(ins)))
    return bases, instrs, data
