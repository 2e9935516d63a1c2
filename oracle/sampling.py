"""Oracle values at sampled points of large grids (test infrastructure only).

A point after T sweeps depends only on inputs within T*r of it, so the FP64
oracle run on that window gives its exact value without stepping the whole
grid; this makes full-size GPU runs checkable point by point.
"""
from __future__ import annotations

import numpy as np

from . import direct


def cone_sample(x0: np.ndarray, w: np.ndarray, steps: int, points, periodic: bool = False,
                binary16: bool = False):
    """Oracle values after `steps` sweeps at the given points of a 1-, 2- or
    3-D grid (points are index tuples), each computed on its dependency cone
    only (FP64 sweeps, or with binary16=True the binary16 sweeps of
    direct.run_binary16, whose roundings act point by point).

    A point after T sweeps depends on inputs within T*r of it along every
    axis.  Running the oracle on that window (clipped to the grid for a zero
    halo) gives the exact value at the window's centre: whatever the window's
    own edges get wrong travels inward at r points per sweep and cannot reach
    the centre in T sweeps.  Periodic grids take the window with wrapped
    indices.
    """
    r = (w.shape[0] - 1) // 2
    reach = steps * r
    step = direct.run_binary16 if binary16 else direct.run
    out = []
    for pt in points:
        if periodic:
            idx = [np.arange(c - reach, c + reach + 1) % n for c, n in zip(pt, x0.shape)]
            win = x0[np.ix_(*idx)].astype(np.float64)
            res = step(win, w, steps, periodic=False)
            out.append(res[(reach,) * x0.ndim])
        else:
            lo = [max(0, c - reach) for c in pt]
            hi = [min(n, c + reach + 1) for c, n in zip(pt, x0.shape)]
            win = x0[tuple(slice(a, b) for a, b in zip(lo, hi))].astype(np.float64)
            res = step(win, w, steps, periodic=False)
            out.append(res[tuple(c - a for c, a in zip(pt, lo))])
    return np.array(out)


def sample_points3(nz: int, ny: int, nx: int, n: int, seed: int = 0):
    """Corners of the box and seeded interior points."""
    pts = [(z, y, x) for z in (0, nz - 1) for y in (0, ny - 1) for x in (0, nx - 1)]
    g = np.random.Generator(np.random.PCG64(seed))
    while len(pts) < n:
        pts.append((int(g.integers(nz)), int(g.integers(ny)), int(g.integers(nx))))
    return pts


def sample_points(ny: int, nx: int, n: int, seed: int = 0):
    """Corners, edge midpoints and seeded interior points."""
    pts = [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1), (ny // 2, 0), (0, nx // 2),
           (ny - 1, nx // 2), (ny // 2, nx - 1)]
    g = np.random.Generator(np.random.PCG64(seed))
    while len(pts) < n:
        pts.append((int(g.integers(ny)), int(g.integers(nx))))
    return pts
