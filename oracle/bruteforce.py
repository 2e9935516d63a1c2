"""Brute-force stencil references for tiny grids (test infrastructure only).

* operator_matrix builds the N x N matrix L of one sweep by visiting every
  (output point, bounding-box offset) pair, so that T sweeps are L^T x.  It
  is written independently of the C stepper and pins it on tiny grids.
* exact_run iterates the definition in exact rational arithmetic (fractions),
  which gives the true result for dyadic coefficients and inputs.
* im2row builds the flattened input matrix B' of stencil flattening
  (Section 3.1) for a 2-D grid with valid-region outputs.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _neighbours(dims, radius, periodic):
    """Yield (output index, offset index in the box, input index or None)."""
    ndim = len(dims)
    k = 2 * radius + 1
    for p in np.ndindex(*dims):
        for o in np.ndindex(*((k,) * ndim)):
            q = []
            inside = True
            for d in range(ndim):
                c = p[d] - radius + o[d]
                if periodic:
                    c %= dims[d]
                elif c < 0 or c >= dims[d]:
                    inside = False
                q.append(c)
            yield p, o, (tuple(q) if inside else None)


def operator_matrix(dims, radius, w, periodic) -> np.ndarray:
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    L = np.zeros((n, n))
    for p, o, q in _neighbours(dims, radius, periodic):
        if q is None:
            continue
        L[np.ravel_multi_index(p, dims), np.ravel_multi_index(q, dims)] += w[o]
    return L


def exact_run(x, radius, w, periodic, steps):
    """T sweeps in exact rational arithmetic; x and w given as floats."""
    dims = x.shape
    cur = {p: Fraction(float(x[p])) for p in np.ndindex(*dims)}
    wf = {o: Fraction(float(w[o])) for o in np.ndindex(*w.shape)}
    for _ in range(steps):
        nxt = {p: Fraction(0) for p in cur}
        for p, o, q in _neighbours(dims, radius, periodic):
            if q is not None:
                nxt[p] += wf[o] * cur[q]
        cur = nxt
    return cur


def im2row(x: np.ndarray, k: int) -> np.ndarray:
    """B' of stencil flattening for valid-region outputs of a 2-D grid:
    column (i, j) (row-major over the (m-k+1) x (n-k+1) outputs) holds the
    k x k window at (i, j) flattened row-major."""
    m, n = x.shape
    cols = []
    for i in range(m - k + 1):
        for j in range(n - k + 1):
            cols.append(x[i:i + k, j:j + k].reshape(-1))
    return np.array(cols).T
