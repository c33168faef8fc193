"""Oracle of the paper's fixed-iteration Jacobi benchmark (TEST
INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may use it).

The "NumPy" section builds the stencil from five views of one array (the
centre and its four shifted neighbours); the "Performance Study" runs it a
fixed number of times on a square array.  Read as an average (each interior
point becomes one fifth of the sum of itself and its four neighbours): with
a coefficient of one on the centre the iteration would grow without bound.
The outermost ring of the array is never written (a fixed boundary).

numpy FP64, whole-array views, no blocking; the sum is taken in the order
centre, up, down, left, right and scaled last.
"""
from __future__ import annotations

import numpy as np


def jacobi5(full: np.ndarray, iters: int) -> np.ndarray:
    """`iters` iterations on a copy of `full` (rows x cols, FP64)."""
    grid = np.array(full, dtype=np.float64, copy=True)
    if grid.ndim != 2:
        raise ValueError("a 2D array is required")
    if grid.shape[0] < 3 or grid.shape[1] < 3:
        return grid  # no interior point
    center = grid[1:-1, 1:-1]
    up = grid[:-2, 1:-1]
    down = grid[2:, 1:-1]
    left = grid[1:-1, :-2]
    right = grid[1:-1, 2:]
    for _ in range(iters):
        work = 0.2 * (center + up + down + left + right)  # all five views read the old values
        center[...] = work
    return grid


def jacobi5_loops(full, iters):
    """The same iteration with explicit loops (small arrays: a brute-force
    check of the view version)."""
    g = [list(map(float, row)) for row in np.asarray(full, dtype=np.float64)]
    rows, cols = len(g), len(g[0])
    for _ in range(iters):
        new = [row[:] for row in g]
        for i in range(1, rows - 1):
            for j in range(1, cols - 1):
                new[i][j] = 0.2 * ((((g[i][j] + g[i - 1][j]) + g[i + 1][j]) + g[i][j - 1]) + g[i][j + 1])
        g = new
    return np.array(g)
