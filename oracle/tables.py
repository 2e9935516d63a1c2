"""Oracle re-derivation of the plan-time tables (test infrastructure only).

Each step follows the paper in its own order and notation, written for
readability rather than speed:

1. bounding_box / compose  -- stencil coefficients as a dense (2r+1)^d array;
   S-fold temporal fusion as the FP64 self-composition of that array
   (Section 4.1 uses 3x temporal fusion without describing the mechanism;
   self-composition, summed in a fixed order, is the reading taken here).
2. morph      -- Adaptive Layout Morphing (Section 3.1): stencil flattening,
   then horizontal crush of r1 adjacent outputs of a row and vertical crush of
   r2 adjacent rows, giving the staircase coefficient matrix A' of
   m' = r1*r2 rows and k' = (k+r1-1)(k+r2-1) columns (Section 3.3).
3. hierarchical_matching -- Algorithm 1 of Section 3.2: block pairs at stride
   s1 = max(floor(m/2), k), then column pairs inside leftover blocks at stride
   s2 = max(floor(g/2), k), zero nodes for what is left, block pairs expanded
   column by column.
4. group      -- pairs of conflict-free columns packed two per 4-wide group,
   zero columns appended up to the fragment's K (Section 3.2: 2:4 as two
   1:2 / 0:2 halves; Section 2.1: sub-2:4 groups are allowed).
5. compress   -- 2 stored values and 2 two-bit positions per row and group
   (Section 3.3, metadata).
6. split_hilo -- coefficient split c = hi + lo/sigma rounded once from FP64.
7. gather_lut -- patch coordinates of every K slot (Section 3.3, lookup table).
8. model      -- layout exploration (Section 3.3, Eqs. 6-11).

Readings where the paper is silent are listed with the function that takes
them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import fpformat

ZETA = -1  # a zero column (the paper's zero node)


# ----------------------------------------------------------------------------
# 1. coefficients

def bounding_box(shape: str, radius: int, ndim: int, coeffs) -> np.ndarray:
    """Dense (2r+1)^ndim float64 coefficient array; star stencils must be
    zero off the axes.  The structural mask used later is the whole box."""
    k = 2 * radius + 1
    w = np.asarray(coeffs, dtype=np.float64).reshape((k,) * ndim)
    if shape == "star":
        for idx in np.ndindex(*w.shape):
            off_axis = sum(1 for i in idx if i != radius)
            if off_axis > 1 and w[idx] != 0.0:
                raise ValueError("star stencil has a coefficient off the axes")
    elif shape != "box":
        raise ValueError(shape)
    return w.copy()


def points_box(offsets, coeffs) -> np.ndarray:
    """Dense box of a stencil given as points (Section 2.2: a pattern of
    neighbours, each with its weight): radius r = the largest |offset
    component| (at least 1), coefficient i at box index offset_i + r, zero
    elsewhere.  A repeated offset is an error."""
    off = np.asarray(offsets, dtype=np.int64)
    c = np.asarray(coeffs, dtype=np.float64).reshape(-1)
    if off.ndim != 2 or off.shape[0] != c.size or off.shape[0] < 1:
        raise ValueError("offsets (npoints, ndim) and one coefficient per point")
    r = max(1, int(np.abs(off).max()))
    w = np.zeros((2 * r + 1,) * off.shape[1])
    seen = set()
    for o, v in zip(off, c):
        key = tuple(int(t) + r for t in o)
        if key in seen:
            raise ValueError("repeated offset")
        seen.add(key)
        w[key] = v
    return w


def compose(w: np.ndarray, steps: int) -> np.ndarray:
    """S-fold composition of a correlation stencil with itself.

    Applying w then v to a periodic grid equals one application of
    c[o] = sum_{a+b=o} w[a] v[b].  The sum for each output offset o (taken in
    row-major order) runs over the first factor's offset a in row-major
    order.  c_S = compose(c_{S-1}, w) with c_{S-1} as the first factor.
    """
    if steps < 1:
        raise ValueError(steps)
    c = w.copy()
    for _ in range(steps - 1):
        c = _compose2(c, w)
    return c


def _compose2(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    ndim = a.ndim
    ka, kb = a.shape[0], b.shape[0]
    kc = ka + kb - 1
    out = np.zeros((kc,) * ndim)
    for o in np.ndindex(*out.shape):
        acc = 0.0
        for ia in np.ndindex(*a.shape):
            ib = tuple(o[d] - ia[d] for d in range(ndim))
            if all(0 <= ib[d] < kb for d in range(ndim)):
                acc += float(a[ia]) * float(b[ib])
        out[o] = acc
    return out


# ----------------------------------------------------------------------------
# 2. Adaptive Layout Morphing

@dataclass(frozen=True)
class MorphDims:
    k: int          # bounding-box width 2r+1
    r1: int         # outputs crushed along x (contiguous)
    r2: int         # output rows crushed along y
    ndim: int
    m_b: int        # row segments per patch plane (k + r2 - 1; 1 in 1-D)
    g: int          # columns per row segment (k + r1 - 1)
    planes: int     # z planes per patch (k in 3-D, else 1)

    @property
    def m_prime(self) -> int:
        return self.r1 * self.r2

    @property
    def k_prime(self) -> int:
        return self.planes * self.m_b * self.g


def morph_dims(k: int, r1: int, r2: int, ndim: int) -> MorphDims:
    if ndim == 1:
        if r2 != 1:
            raise ValueError("1-D layouts have r2 = 1")
        return MorphDims(k, r1, 1, 1, 1, k + r1 - 1, 1)
    planes = k if ndim == 3 else 1
    return MorphDims(k, r1, r2, ndim, k + r2 - 1, k + r1 - 1, planes)


def morph(w: np.ndarray, r1: int, r2: int):
    """Staircase matrix A' (m' x k') and its structural mask.

    Row ty*r1 + tx is output (ty, tx) of an r2 x r1 tile; column
    (pz*m_b + pr)*g + pc is patch element (pz, pr, pc) of the tile's halo'd
    input patch.  Horizontal crush expands each kernel row into r1 rows with a
    one-column shift per row; vertical crush shifts by one row segment per
    output row: A'[(ty,tx), (pz,pr,pc)] = w[pz][pr-ty][pc-tx] when both
    differences lie in [0, k).  The structure is the whole bounding box.
    """
    ndim = w.ndim
    k = w.shape[0]
    d = morph_dims(k, r1, r2, ndim)
    a = np.zeros((d.m_prime, d.k_prime))
    s = np.zeros((d.m_prime, d.k_prime), dtype=bool)
    for ty in range(d.r2):
        for tx in range(d.r1):
            row = ty * r1 + tx
            for pz in range(d.planes):
                for pr in range(d.m_b):
                    for pc in range(d.g):
                        col = (pz * d.m_b + pr) * d.g + pc
                        a_ = pc - tx
                        if ndim == 1:
                            if 0 <= a_ < k:
                                a[row, col] = w[a_]
                                s[row, col] = True
                            continue
                        b_ = pr - ty
                        if 0 <= a_ < k and 0 <= b_ < k:
                            s[row, col] = True
                            a[row, col] = w[b_, a_] if ndim == 2 else w[pz, b_, a_]
    return a, s, d


def patch_coords(d: MorphDims, col: int):
    """(pz, pr, pc) of a column of A'."""
    pz, rem = divmod(col, d.m_b * d.g)
    pr, pc = divmod(rem, d.g)
    return pz, pr, pc


# ----------------------------------------------------------------------------
# 3. Algorithm 1 (hierarchical two-level matching)

def hierarchical_matching(m: int, g: int, k: int):
    """Algorithm 1 on one staircase plane of m blocks of g columns.

    Returns (pairs, zeros): a list of ((block, col), (block, col) | None) in
    the order the algorithm builds them (block pairs expanded column by
    column first, then the in-block pairs), and the number of zero nodes.

    Written from what the two levels produce rather than as a loop:

    * level 1 pairs whole blocks s1 = max(floor(m/2), k) apart (Theorem 1:
      they share no output row).  Scanning blocks upward and pairing each
      free block with the one s1 above it, the pairs are (i, i + s1) for the
      blocks i that are below s1 (a block at or above s1 is already someone's
      partner) and have a block s1 above them (i + s1 < m);
    * level 2 works on each block no level-1 pair covers: columns
      s2 = max(floor(g/2), k) apart never share an output row, so the same
      scan pairs (u, u + s2) for u < s2 with u + s2 < g; a column in
      neither role gets a zero node.

    The sets are formed first and then listed in the paper's order (M1
    expanded over the g columns of each block pair, then M2 by block and
    source column); every column of the plane must appear exactly once.
    """
    s1 = max(m // 2, k)
    m1 = [(i, i + s1) for i in range(m) if i < s1 and i + s1 < m]
    covered = {b for pair in m1 for b in pair}
    s2 = max(g // 2, k)
    sources = {u for u in range(g) if u < s2 and u + s2 < g}
    targets = {u + s2 for u in sources}
    singles = set(range(g)) - sources - targets
    m2 = []
    zeros = 0
    for x in sorted(set(range(m)) - covered):
        for u in sorted(sources | singles):
            if u in sources:
                m2.append(((x, u), (x, u + s2)))
            else:
                m2.append(((x, u), None))
                zeros += 1
    pairs = [((p, t), (q, t)) for p, q in m1 for t in range(g)]
    pairs.extend(m2)
    seen = [c for a, b in pairs for c in (a, b) if c is not None]
    assert len(seen) == len(set(seen)) == m * g
    return pairs, zeros


def plane_pairs(d: MorphDims):
    """Column-index pairs for the whole of A' (planes concatenated in order).

    In 3-D every output row uses every plane, so planes never pair with each
    other; Algorithm 1 runs on each plane's block staircase.  In 1-D the plane
    is a single block.  Returns (pairs, zeros) with ZETA for zero nodes."""
    base, zeros = hierarchical_matching(d.m_b, d.g, d.k)
    out = []
    for pz in range(d.planes):
        off = pz * d.m_b * d.g
        for a, b in base:
            ca = off + a[0] * d.g + a[1]
            cb = ZETA if b is None else off + b[0] * d.g + b[1]
            out.append((ca, cb))
    return out, zeros * d.planes


def thm2_zero_count(d: MorphDims) -> int:
    """Zero nodes predicted per plane by the argument of Theorem 2: unmatched
    blocks times the zero nodes of one local graph."""
    s1 = max(d.m_b // 2, d.k)
    s2 = max(d.g // 2, d.k)
    u_b = d.m_b - 2 * min(max(d.m_b - s1, 0), s1)
    z_loc = d.g - 2 * min(max(d.g - s2, 0), s2)
    return u_b * z_loc * d.planes


# ----------------------------------------------------------------------------
# 4. grouping into 4-wide groups and padding to the fragment K

def group(pairs, kfrag: int):
    """perm[K_pad]: A' column feeding each K slot (ZETA for a zero column).

    Reading (the paper does not fix the packing): consecutive pairs P0, P1
    form one group laid out as [P0.a, P1.a, P0.b, P1.b]; an odd pair count gets
    one (zero, zero) pair; (zero, zero) pairs are appended until the column
    count is a multiple of kfrag.  Any order inside a group of two
    conflict-free pairs is 2:4-valid; this one puts the column-t and
    column-(t+1) elements of a block pair next to each other."""
    ps = list(pairs)
    if len(ps) % 2:
        ps.append((ZETA, ZETA))
    while (2 * len(ps)) % kfrag:
        ps.append((ZETA, ZETA))
    perm = []
    for j in range(0, len(ps), 2):
        p0, p1 = ps[j], ps[j + 1]
        perm.extend([p0[0], p1[0], p0[1], p1[1]])
    return perm


def conflict(s: np.ndarray, i: int, j: int) -> bool:
    """Definition 1: columns i, j conflict iff some row is nonzero in both."""
    if i == ZETA or j == ZETA:
        return False
    return bool(np.any(s[:, i] & s[:, j]))


# ----------------------------------------------------------------------------
# 5. compression with metadata

def compress(a: np.ndarray, s: np.ndarray, perm):
    """Per row and 4-group: two stored values and their positions (i0 < i1).

    The structural positions of the group (at most two, or the group is
    invalid) are kept; if fewer than two, the smallest unused positions fill
    up the pair (sub-2:4 groups, Section 2.1).  Values at fillers and zero
    columns are 0.  Returns values (m' x K_pad/2) and meta (m' x K_pad/4 x 2).
    """
    mp = a.shape[0]
    kp = len(perm)
    vals = np.zeros((mp, kp // 2))
    meta = np.zeros((mp, kp // 4, 2), dtype=np.int64)
    for i in range(mp):
        for j in range(kp // 4):
            cols = perm[4 * j: 4 * j + 4]
            live = [p for p in range(4) if cols[p] != ZETA and s[i, cols[p]]]
            if len(live) > 2:
                raise ValueError(f"row {i} group {j} holds {len(live)} nonzeros")
            fill = [p for p in range(4) if p not in live]
            pos = sorted(live + fill[: 2 - len(live)])
            for t, p in enumerate(pos):
                meta[i, j, t] = p
                vals[i, 2 * j + t] = a[i, cols[p]] if (cols[p] != ZETA and s[i, cols[p]]) else 0.0
    return vals, meta


def permuted(a: np.ndarray, perm) -> np.ndarray:
    """A'' = A' with columns permuted by perm (zero columns for ZETA)."""
    out = np.zeros((a.shape[0], len(perm)))
    for kk, c in enumerate(perm):
        if c != ZETA:
            out[:, kk] = a[:, c]
    return out


# ----------------------------------------------------------------------------
# 6. hi/lo split of the coefficients

SIGMA = {"f16": 2.0 ** 11, "bf16": 1.0}


def split_hilo(vals: np.ndarray, fmt: str):
    """c_hi = RNE(c), c_lo = RNE(sigma * (c - c_hi)), both rounded once from
    FP64.  Returns uint16 bit patterns (hi, lo).  Overflow raises."""
    spec = fpformat.BINARY16 if fmt == "f16" else fpformat.BFLOAT16
    bits = fpformat.f16_bits if fmt == "f16" else fpformat.bf16_bits
    sigma = SIGMA[fmt]
    hi = np.zeros(vals.shape, dtype=np.uint16)
    lo = np.zeros(vals.shape, dtype=np.uint16)
    for idx in np.ndindex(*vals.shape):
        c = float(vals[idx])
        h = fpformat.round_rne(c, spec)
        if h is None:
            raise OverflowError(c)
        l_ = fpformat.round_rne(sigma * (c - h), spec)
        if l_ is None:
            raise OverflowError(c)
        hi[idx] = bits(h)
        lo[idx] = bits(l_)
    return hi, lo


def split_three_bf16(vals: np.ndarray):
    """Three-part bfloat16 split of FP64 coefficients: c_hi = RNE(c), c_mid =
    RNE(c - c_hi), c_lo = RNE(c - c_hi - c_mid), each rounded once from the
    exact FP64 remainder.  Returns uint16 bit patterns (hi, mid, lo)."""
    spec = fpformat.BFLOAT16
    out = [np.zeros(vals.shape, dtype=np.uint16) for _ in range(3)]
    for idx in np.ndindex(*vals.shape):
        r = float(vals[idx])
        for t in range(3):
            v = fpformat.round_rne(r, spec)
            if v is None:
                raise OverflowError(float(vals[idx]))
            out[t][idx] = fpformat.bf16_bits(v)
            r -= v
    return tuple(out)


def round_plain(vals: np.ndarray, fmt: str) -> np.ndarray:
    """Single-part rounding (plain FP16/BF16 paths): uint16 bit patterns."""
    spec = fpformat.BINARY16 if fmt == "f16" else fpformat.BFLOAT16
    bits = fpformat.f16_bits if fmt == "f16" else fpformat.bf16_bits
    out = np.zeros(vals.shape, dtype=np.uint16)
    for idx in np.ndindex(*vals.shape):
        h = fpformat.round_rne(float(vals[idx]), spec)
        if h is None:
            raise OverflowError(float(vals[idx]))
        out[idx] = bits(h)
    return out


# ----------------------------------------------------------------------------
# 7. gather lookup table

def gather_lut(d: MorphDims, perm):
    """(pz, pr, pc) of the patch element feeding each K slot; (-1,-1,-1) for
    zero columns."""
    out = np.full((len(perm), 3), -1, dtype=np.int64)
    for kk, c in enumerate(perm):
        if c != ZETA:
            out[kk] = patch_coords(d, c)
    return out


# ----------------------------------------------------------------------------
# 7b. structure-aware K orders of the kernels (beyond the paper)
#
# The paper's structure is the bounding box, so a star stencil's never-used
# patch columns still occupy K.  This build's reading for the kernels: a
# column is used when some row of A' holds a nonzero value in it.  Sparse
# order: walk Algorithm 1's groups; each group is two dominoes (slots 0-1 and
# 2-3, horizontally adjacent columns feeding one 32-bit B register).  Keep a
# group when both dominoes hold a used column, drop it when neither does,
# otherwise set its used domino aside.  Then, in the order they were set
# aside, give each unpaired domino the first later unpaired domino whose
# columns share no nonzero row with its own, position by position (the two
# halves of the new group are then Definition-1 conflict-free pairs), or a
# domino of zero columns.  Kept groups come first, new groups after, zero
# columns up to the fragment's K.  Dense order: the natural column order in
# pairs (c, c+1), c even, keeping the pairs that hold a used column, zero
# columns up to the fragment's K.

def used_columns(a: np.ndarray) -> np.ndarray:
    """Columns of A' with a nonzero value in some row."""
    return np.array([bool(np.count_nonzero(a[:, c])) for c in range(a.shape[1])])


def _kept_and_aside(a: np.ndarray, perm, g: int):
    """Algorithm 1's 4-groups both of whose halves hold a used column (and,
    with g even, are aligned dominoes), kept in order; and the used dominoes
    set aside for re-pairing: the used halves of half-used groups, and the
    aligned dominoes (pc, pc + 1), pc even, of the columns of groups with a
    half that is not one (each once, in order of first appearance)."""
    used = used_columns(a)
    aligned_only = g > 0 and g % 2 == 0

    def holds_used(domino):
        return any(c != ZETA and used[c] for c in domino)

    def aligned(half):
        if half == (ZETA, ZETA):
            return True
        c0, c1 = half
        return c0 != ZETA and c1 == c0 + 1 and (c0 % g) % 2 == 0

    kept, aside, seen = [], [], set()
    for j in range(0, len(perm), 4):
        first, second = tuple(perm[j:j + 2]), tuple(perm[j + 2:j + 4])
        if aligned_only and not (aligned(first) and aligned(second)):
            for c in perm[j:j + 4]:
                if c == ZETA:
                    continue
                d0 = c - (c % g) % 2
                if d0 not in seen:
                    seen.add(d0)
                    if holds_used((d0, d0 + 1)):
                        aside.append((d0, d0 + 1))
            continue
        u1, u2 = holds_used(first), holds_used(second)
        if u1 and u2:
            kept.append(list(perm[j:j + 4]))
        elif u1:
            aside.append(first)
        elif u2:
            aside.append(second)
    return kept, aside


def dominoes_compatible(a: np.ndarray, d0, d1) -> bool:
    """Two dominoes may share a 4-group [d0.0, d0.1, d1.0, d1.1]: their
    first columns, and their second columns, are conflict-free pairs
    (Definition 1 on the nonzeros of A')."""
    def rows_of(c):
        return set() if c == ZETA else set(np.flatnonzero(a[:, c]))
    return not (rows_of(d0[0]) & rows_of(d1[0])) and not (rows_of(d0[1]) & rows_of(d1[1]))


def compact_sparse_order(a: np.ndarray, perm, kfrag: int, g: int = 0):
    """Kernel K order: Algorithm 1's 4-groups with the columns the stencil
    never uses dropped and half-used groups re-paired first fit (each
    set-aside domino with the first later compatible one).

    With g (the patch row length, even) given, every half of a kept group is
    also a horizontal domino (pc, pc + 1) with pc even: the columns of any
    group with another half are taken apart into such dominoes, which join
    the re-pairing (_kept_and_aside)."""
    kept, aside = _kept_and_aside(a, perm, g)
    paired = [False] * len(aside)
    new = []
    for i, dom in enumerate(aside):
        if paired[i]:
            continue
        paired[i] = True
        partner = (ZETA, ZETA)
        for j in range(i + 1, len(aside)):
            if not paired[j] and dominoes_compatible(a, dom, aside[j]):
                partner = aside[j]
                paired[j] = True
                break
        new.append([dom[0], dom[1], partner[0], partner[1]])
    out = [c for grp in kept + new for c in grp]
    while len(out) % kfrag:
        out.append(ZETA)
    return out


def max_repairing_groups(a: np.ndarray, perm, g: int):
    """(kept groups, least number of groups the set-aside dominoes fit in):
    the re-pairing as a maximum matching of the compatibility graph of the
    dominoes (networkx's general-graph matching, independent of the
    planner's)."""
    import networkx as nx
    kept, aside = _kept_and_aside(a, perm, g)
    graph = nx.Graph()
    graph.add_nodes_from(range(len(aside)))
    for i in range(len(aside)):
        for j in range(i + 1, len(aside)):
            if dominoes_compatible(a, aside[i], aside[j]):
                graph.add_edge(i, j)
    matching = nx.max_weight_matching(graph, maxcardinality=True)
    return kept, len(aside) - len(matching)


def compact_dense_order(a: np.ndarray, kfrag: int):
    used = used_columns(a)
    kp = a.shape[1]
    out = []
    for c in range(0, kp, 2):
        pair = [c, c + 1 if c + 1 < kp else ZETA]
        if any(x != ZETA and used[x] for x in pair):
            out.extend(pair)
    while len(out) % kfrag:
        out.append(ZETA)
    return out


# ----------------------------------------------------------------------------
# 8. layout exploration model (Section 3.3, Eqs. 6-11)

@dataclass(frozen=True)
class Machine:
    """Constants of the analytical model for one MI355X (spec values)."""
    freq_hz: float = 2.4e9
    n_tcu: int = 1024              # 256 CUs x 4 matrix cores
    cpi_mma: float = 16.0          # cycles of one 16x16x64 sparse / 16x16x32 dense f16 op
    bw_global: float = 8.0e12      # HBM bytes/s
    bw_shared: float = 256 * 128 * 2.4e9  # LDS bytes/s (128 B/clk/CU)
    frag_m: int = 16
    frag_n: int = 16
    frag_k: int = 64


def model_time(k: int, ndim: int, r1: int, r2: int, grid, elem_bytes: int,
               coef_bytes: int, passes: int, planes_state: int, mach: Machine = Machine()):
    """T = max(T_compute, T_memory) for one layout candidate.

    N_MMA = ceil(m'/M) ceil(k''/K) ceil(n'/N) (Eq. 9) with k'' the column
    count after sparsity conversion and n' the number of tiles covering the
    grid; T_compute = N_MMA * passes * CPI / (f * N_tcu) (Eq. 7); T_memory =
    max(global read+write / bw_G, shared read+write / bw_S) (Eq. 8) with
    data_transR = data_transW = k'(m'/2 + n') elements (Eq. 10, reading the
    garbled 'm/2' as m'/2 because A' is stored compressed to half its width).
    Returns (T, T_compute, T_global, T_shared, K_pad).
    """
    d = morph_dims(k, r1, r2, ndim)
    pairs, _z = plane_pairs(d)
    perm = group(pairs, mach.frag_k)
    kpad = len(perm)
    if ndim == 1:
        n_tiles = math.ceil(grid[0] / r1)
        points = grid[0]
    elif ndim == 2:
        n_tiles = math.ceil(grid[0] / r2) * math.ceil(grid[1] / r1)
        points = grid[0] * grid[1]
    else:
        n_tiles = grid[0] * math.ceil(grid[1] / r2) * math.ceil(grid[2] / r1)
        points = grid[0] * grid[1] * grid[2]
    n_mma = (math.ceil(d.m_prime / mach.frag_m) * math.ceil(kpad / mach.frag_k)
             * math.ceil(n_tiles / mach.frag_n))
    t_compute = n_mma * passes * mach.cpi_mma / (mach.freq_hz * mach.n_tcu)
    data_r = points * elem_bytes * planes_state
    data_w = points * elem_bytes * planes_state
    t_global = (data_r + data_w) / mach.bw_global
    trans = d.k_prime * (d.m_prime / 2.0 + n_tiles)
    trans_r = trans * coef_bytes * passes_planes(passes)
    trans_w = trans_r
    t_shared = (trans_r + trans_w) / mach.bw_shared
    t = max(t_compute, max(t_global, t_shared))
    return t, t_compute, t_global, t_shared, kpad


def passes_planes(passes: int) -> int:
    """Parts of the operands moved through LDS: hi and lo in split mode
    (three products), hi, mid and lo with three parts (six products)."""
    return 3 if passes >= 6 else 2 if passes > 1 else 1


def explore(k: int, ndim: int, grid, candidates, elem_bytes: int, coef_bytes: int,
            passes: int, planes_state: int, mach: Machine = Machine()):
    """Eq. 11: argmin of T over the candidate set.

    Reading of the tie-break (the paper gives none): smallest T (relative
    tolerance 1e-12); then smallest T_compute (the matrix work, which is
    what separates layouts that tie on an HBM-bound T); then smallest
    T_shared; then smaller K_pad; then smaller r1*r2; then smaller r1.  Returns
    ((r1, r2), table) with table[(r1, r2)] = model_time(...)."""
    table = {}
    for (r1, r2) in candidates:
        table[(r1, r2)] = model_time(k, ndim, r1, r2, grid, elem_bytes, coef_bytes,
                                     passes, planes_state, mach)
    best = None
    for c in candidates:
        if best is None or _better(table[c], c, table[best], best):
            best = c
    return best, table


def _better(ta, ca, tb, cb) -> bool:
    def close(x, y):
        return abs(x - y) <= 1e-12 * max(abs(x), abs(y))
    if not close(ta[0], tb[0]):
        return ta[0] < tb[0]
    if not close(ta[1], tb[1]):
        return ta[1] < tb[1]
    if not close(ta[3], tb[3]):
        return ta[3] < tb[3]
    if ta[4] != tb[4]:
        return ta[4] < tb[4]
    if ca[0] * ca[1] != cb[0] * cb[1]:
        return ca[0] * ca[1] < cb[0] * cb[1]
    return ca[0] < cb[0]
