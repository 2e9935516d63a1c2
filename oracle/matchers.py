"""Exhaustive validators for the structured-sparsity conversion (test only).

These solve the paper's optimisation problems by plain search on small
shapes, independently of Algorithm 1:

* min_zero_pairing -- Problem 1 (Section 3.2): the least number p of zero
  columns such that the columns of A', plus p zero columns, split into
  conflict-free pairs (Definitions 1-3).  Equivalently k' minus twice a
  maximum matching of the complement of the conflict graph.
* min_pad_groups   -- the exact 2:4 question: the least number of zero
  columns such that the columns split into groups of 4 with at most 2
  structural nonzeros per row in each group (Eq. 2), with pads counted up to
  a multiple of 4.

Both use memoised search that always branches on the lowest unplaced
column, which keeps them exact; they are meant for k' up to about 24-40.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np


def conflict_matrix(s: np.ndarray) -> np.ndarray:
    """c[i, j] = True iff columns i and j share a structurally nonzero row."""
    si = s.astype(np.int64)
    return (si.T @ si) > 0


def min_zero_pairing(s: np.ndarray) -> int:
    c = conflict_matrix(s)
    n = c.shape[0]
    compat = [0] * n
    for i in range(n):
        for j in range(n):
            if i != j and not c[i, j]:
                compat[i] |= 1 << j
    full = (1 << n) - 1

    @lru_cache(maxsize=None)
    def best(mask: int) -> int:
        # maximum number of pairs among the columns in mask
        if mask == 0:
            return 0
        i = (mask & -mask).bit_length() - 1
        rest = mask & ~(1 << i)
        res = best(rest)                 # column i goes with a zero column
        cand = compat[i] & rest
        while cand:
            j = (cand & -cand).bit_length() - 1
            cand &= cand - 1
            v = 1 + best(rest & ~(1 << j))
            if v > res:
                res = v
        return res

    return n - 2 * best(full)


def group_ok(s: np.ndarray, cols) -> bool:
    """At most two structural nonzeros per row among the given columns."""
    if not cols:
        return True
    return bool(np.all(s[:, list(cols)].sum(axis=1) <= 2))


def min_pad_groups(s: np.ndarray) -> int:
    n = s.shape[1]
    rows_of = [int(sum(1 << r for r in range(s.shape[0]) if s[r, c])) for c in range(n)]

    def ok(cols) -> bool:
        # at most two columns of the group share any row
        for r in range(s.shape[0]):
            cnt = 0
            for c in cols:
                if rows_of[c] >> r & 1:
                    cnt += 1
            if cnt > 2:
                return False
        return True

    @lru_cache(maxsize=None)
    def best(mask: int) -> int:
        # least pads to group the columns of mask into valid groups of 4
        if mask == 0:
            return 0
        i = (mask & -mask).bit_length() - 1
        rest = mask & ~(1 << i)
        others = [j for j in range(n) if rest >> j & 1]
        res = 3 + best(rest)  # i alone with three pads
        for a in range(len(others)):
            ca = others[a]
            if not ok((i, ca)):
                continue
            res = min(res, 2 + best(rest & ~(1 << ca)))
            for b in range(a + 1, len(others)):
                cb = others[b]
                if not ok((i, ca, cb)):
                    continue
                m2 = rest & ~(1 << ca) & ~(1 << cb)
                res = min(res, 1 + best(m2))
                for c_ in range(b + 1, len(others)):
                    cc = others[c_]
                    if ok((i, ca, cb, cc)):
                        res = min(res, best(m2 & ~(1 << cc)))
        return res

    return best((1 << n) - 1)
