"""Oracle values at sampled points of large grids (test infrastructure only).

A point after T sweeps depends only on inputs within T*r of it, so the FP64
oracle run on that window gives its exact value without stepping the whole
grid; this makes full-size GPU runs checkable point by point.
"""
from __future__ import annotations

import numpy as np

from . import direct


def cone_sample(x0: np.ndarray, w: np.ndarray, steps: int, points, periodic: bool = False):
    """Oracle values after `steps` sweeps at the given points of a 2-D grid,
    each computed on its dependency cone only.

    A point after T sweeps depends on inputs within T*r of it.  Running the
    oracle on that window (clipped to the grid for a zero halo) gives the exact
    value at the window's centre: whatever the window's own edges get wrong
    travels inward at r points per sweep and cannot reach the centre in T
    sweeps.  Periodic grids take the window with wrapped indices.
    """
    r = (w.shape[0] - 1) // 2
    ny, nx = x0.shape
    reach = steps * r
    out = []
    for (y, x) in points:
        if periodic:
            ys = np.arange(y - reach, y + reach + 1) % ny
            xs = np.arange(x - reach, x + reach + 1) % nx
            win = x0[np.ix_(ys, xs)].astype(np.float64)
            res = direct.run(win, w, steps, periodic=False)
            out.append(res[reach, reach])
        else:
            y0, y1 = max(0, y - reach), min(ny, y + reach + 1)
            x0_, x1 = max(0, x - reach), min(nx, x + reach + 1)
            win = x0[y0:y1, x0_:x1].astype(np.float64)
            res = direct.run(win, w, steps, periodic=False)
            out.append(res[y - y0, x - x0_])
    return np.array(out)


def sample_points(ny: int, nx: int, n: int, seed: int = 0):
    """Corners, edge midpoints and seeded interior points."""
    pts = [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1), (ny // 2, 0), (0, nx // 2),
           (ny - 1, nx // 2), (ny // 2, nx - 1)]
    g = np.random.Generator(np.random.PCG64(seed))
    while len(pts) < n:
        pts.append((int(g.integers(ny)), int(g.integers(nx))))
    return pts
