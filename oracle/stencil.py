"""Oracle of the synthetic stencil workload (TEST INFRASTRUCTURE ONLY: the
tests, the smoke check and the benchmark's CPU baseline may use it).

The paper's performance study runs "a synthetic stencil simulation" that
relies on NumPy slicing, on 10240 x 1024 elements for 10 time steps, without
stating the stencil (parity of the stencil itself with the paper is
therefore unpinned).  Reading taken here: each step replaces every interior
point by the mean of its 3 x 3 neighbourhood, computed from the previous
step's values (nine views of the array), the outermost ring held fixed; the
nine values are summed in row-major neighbourhood order (north-west first,
south-east last) and divided by 9.

numpy FP64, whole-array views, no blocking.
"""
from __future__ import annotations

import numpy as np

# (row, column) offsets of the nine views, in summation order
NEIGHBOURS = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 0), (0, 1), (1, -1), (1, 0), (1, 1)]


def stencil9(full: np.ndarray, steps: int) -> np.ndarray:
    """`steps` time steps on a copy of `full` (rows x cols, FP64)."""
    a = np.array(full, dtype=np.float64, copy=True)
    if a.ndim != 2:
        raise ValueError("a 2D array is required")
    R, C = a.shape
    if R < 3 or C < 3:
        return a
    b = a.copy()
    for _ in range(steps):
        views = [a[1 + di:R - 1 + di, 1 + dj:C - 1 + dj] for di, dj in NEIGHBOURS]
        s = views[0] + views[1]
        for v in views[2:]:
            s = s + v
        b[1:-1, 1:-1] = s / 9.0
        a, b = b, a
    return a


def stencil9_loops(full, steps):
    """The same with explicit loops (small arrays: a brute-force check)."""
    g = [list(map(float, row)) for row in np.asarray(full, dtype=np.float64)]
    R, C = len(g), len(g[0])
    for _ in range(steps):
        new = [row[:] for row in g]
        for i in range(1, R - 1):
            for j in range(1, C - 1):
                s = g[i - 1][j - 1]
                for di, dj in NEIGHBOURS[1:]:
                    s = s + g[i + di][j + dj]
                new[i][j] = s / 9.0
        g = new
    return np.array(g)
