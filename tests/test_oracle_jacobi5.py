"""Pins of the oracle of the paper's fixed-iteration Jacobi benchmark
(five-view average, fixed boundary): brute force, the C oracle's weighted
Jacobi, exact eigenvalues on a rectangle, fixed points and the maximum
principle."""
import numpy as np
import pytest

import oracle as O
from oracle.jacobi5 import jacobi5, jacobi5_loops
from paper_1210_7774_amd import inputs as I


@pytest.mark.parametrize("shape,iters", [((9, 13), 0), ((9, 13), 1), ((9, 13), 5), ((3, 3), 2), ((4, 11), 3),
                                         ((2, 7), 2), ((1, 1), 1)])
def test_views_match_loops_bitwise(shape, iters):
    x = I.uniform_field(shape, 8)
    assert np.array_equal(jacobi5(x, iters), jacobi5_loops(x, iters))


def test_zero_boundary_is_weighted_jacobi():
    """With a zero ring and f = 0 the iteration is the C oracle's weighted
    Jacobi with omega = 4/5 on the interior (independent code)."""
    rows, cols = 19, 19  # the C oracle's grids are square
    x = I.uniform_field((rows, cols), 9)
    x[0, :] = x[-1, :] = x[:, 0] = x[:, -1] = 0.0
    got = jacobi5(x, 6)
    u = np.ascontiguousarray(x[1:-1, 1:-1]).copy()
    for _ in range(6):
        O.sweep(u, np.zeros_like(u), kind=O.JACOBI, omega=0.8)
    assert np.abs(got[1:-1, 1:-1] - u).max() <= 1e-14
    assert not np.any(got[0, :]) and not np.any(got[:, 0])


@pytest.mark.parametrize("k,l", [(1, 2), (3, 1), (5, 4)])
def test_eigenmode_on_rectangle(k, l):
    """sin(k pi i/(R-1)) sin(l pi j/(C-1)) with a zero ring is multiplied by
    0.2 (1 + 2 cos(k pi/(R-1)) + 2 cos(l pi/(C-1))) per iteration; R != C
    and k != l catch swapped axes."""
    R, C = 17, 29
    i = np.arange(R)[:, None]
    j = np.arange(C)[None, :]
    m = np.sin(k * np.pi * i / (R - 1)) * np.sin(l * np.pi * j / (C - 1))
    lam = 0.2 * (1 + 2 * np.cos(k * np.pi / (R - 1)) + 2 * np.cos(l * np.pi / (C - 1)))
    for t in (1, 4):
        assert np.abs(jacobi5(m, t) - lam ** t * m).max() <= 1e-14


def test_fixed_points_and_boundary():
    R, C = 12, 21
    i = np.arange(R)[:, None] * np.ones((1, C))
    j = np.arange(C)[None, :] * np.ones((R, 1))
    lin = 0.5 + 0.25 * i - 0.125 * j  # discrete harmonic: a fixed point
    assert np.abs(jacobi5(lin, 7) - lin).max() <= 1e-13
    const = np.full((R, C), 3.0)
    assert np.abs(jacobi5(const, 4) - const).max() <= 1e-14
    x = I.uniform_field((R, C), 10)
    y = jacobi5(x, 4)
    ring = np.ones((R, C), bool)
    ring[1:-1, 1:-1] = False
    assert np.array_equal(y[ring], x[ring])
    assert np.array_equal(jacobi5(x, 0), x)
    # maximum principle: an average never leaves the data's range
    assert y.min() >= x.min() and y.max() <= x.max()


def test_planted_mistakes_fail():
    """A dropped neighbour, a coefficient on the centre of one, or a swapped
    axis each break one of the pins above (checked on the CPU here)."""
    R, C = 17, 29
    i = np.arange(R)[:, None]
    j = np.arange(C)[None, :]
    m = np.sin(np.pi * i / (R - 1)) * np.sin(2 * np.pi * j / (C - 1))
    lam = 0.2 * (1 + 2 * np.cos(np.pi / (R - 1)) + 2 * np.cos(2 * np.pi / (C - 1)))

    def variant(g, kind):
        g = g.copy()
        c, u, d, lf, rt = g[1:-1, 1:-1], g[:-2, 1:-1], g[2:, 1:-1], g[1:-1, :-2], g[1:-1, 2:]
        if kind == "drop":
            w = 0.2 * (c + u + d + lf)
        elif kind == "printed":
            w = c + 0.2 * (u + d + lf + rt)
        else:  # a square-grid eigenvalue used on the rectangle: axes mixed up
            w = 0.2 * (c + u + d + lf + rt)
            return np.abs(w - (0.2 * (1 + 2 * np.cos(2 * np.pi / (R - 1)) + 2 * np.cos(np.pi / (C - 1))))
                          * c).max()
        g[1:-1, 1:-1] = w
        return np.abs(g - lam * m).max()

    for kind in ("drop", "printed", "swap"):
        assert variant(m, kind) > 1e-3, kind
