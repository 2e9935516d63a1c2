"""Pins of the oracle's plan-time tables (oracle/tables.py) against what the
paper fixes: the morph dimensions (Section 3.3), the duplicate relations
Eq. 3 / Eq. 4 and exact reproduction of the stencil by A' times the crushed
patches (Section 3.1), PIT invariance (Eq. 5), Theorem 1 (conflict freedom),
Theorem 2 (zero count, per-subgraph optimality checked by exhaustive search),
lossless compression with metadata, the split error bounds, and the
layout-exploration model (Eqs. 6-11) against hand-computed values."""
import json
import math
import os

import numpy as np
import pytest

import synthetic
from oracle import bruteforce, direct, fpformat, matchers
from oracle import tables as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

SHAPES_2D = [(3, 8, 8), (3, 4, 4), (3, 8, 2), (3, 16, 1), (3, 16, 4), (7, 8, 8), (7, 16, 4),
             (7, 16, 1), (13, 8, 8), (13, 16, 4), (5, 16, 1), (3, 2, 2), (3, 3, 2), (5, 2, 2),
             (3, 5, 1), (3, 7, 2), (3, 32, 4), (5, 8, 8), (9, 8, 8), (11, 16, 4)]


@pytest.mark.parametrize("k,r1,r2", SHAPES_2D)
def test_morph_dimensions_closed_form(k, r1, r2):
    # Section 3.3: m' = r1 r2 and k' = (k + r1 - 1)(k + r2 - 1).
    w = np.ones((k, k))
    a, s, d = T.morph(w, r1, r2)
    assert a.shape == (r1 * r2, (k + r1 - 1) * (k + r2 - 1))
    # every output row uses exactly k^2 structural entries (one per kernel element)
    assert np.all(s.sum(axis=1) == k * k)


def test_morph_dimensions_3d_and_1d():
    a, s, d = T.morph(np.ones((3, 3, 3)), 8, 8)
    assert a.shape == (64, 3 * 100)
    a, s, d = T.morph(np.ones(5), 16, 1)
    assert a.shape == (16, 20)


def test_duplicate_relations_eq3_eq4():
    # B_a[b, (y, x)] = X[y+a][x+b] for kernel row a, column b (Section 3.1).
    g = synthetic.rng(21)
    m, n, k = 9, 11, 3
    X = g.integers(-50, 50, size=(m, n)).astype(np.float64)
    Bp = bruteforce.im2row(X, k)
    nx = n - k + 1
    ny = m - k + 1

    def B(a, b, y, x):
        return Bp[a * k + b, y * nx + x]
    for a in range(k):
        for b in range(k - 1):
            for y in range(ny):
                for x in range(nx - 1):
                    assert B(a, b + 1, y, x) == B(a, b, y, x + 1)           # Eq. 3
    for a in range(k - 1):
        for b in range(k):
            for y in range(ny - 1):
                for x in range(nx):
                    assert B(a + 1, b, y, x) == B(a, b, y + 1, x)           # Eq. 4


@pytest.mark.parametrize("k,r1,r2", [(3, 8, 8), (3, 4, 2), (5, 4, 4), (7, 8, 8), (3, 3, 2)])
def test_crushed_product_equals_flattened_product(k, r1, r2):
    # Stencil flattening gives out = W_flat . B'; after both crushes the same
    # outputs come from A' times the crushed patch, exactly on integer data.
    g = synthetic.rng(22)
    w = g.integers(-4, 5, size=(k, k)).astype(np.float64)
    a, s, d = T.morph(w, r1, r2)
    m, n = 3 * r2 + k - 1, 2 * r1 + k - 1
    X = g.integers(-20, 21, size=(m, n)).astype(np.float64)
    flat = w.reshape(-1) @ bruteforce.im2row(X, k)
    flat = flat.reshape(m - k + 1, n - k + 1)
    for y0 in range(0, m - k + 1, r2):
        for x0 in range(0, n - k + 1, r1):
            patch = X[y0:y0 + d.m_b, x0:x0 + d.g].reshape(-1)
            out = (a @ patch).reshape(r2, r1)
            assert np.array_equal(out, flat[y0:y0 + r2, x0:x0 + r1])


def padded_patch(X, d, origin, radius):
    """Halo'd patch of a tile with zeros outside the grid (any ndim)."""
    ndim = X.ndim
    if ndim == 1:
        idx = [origin[0] - radius + pc for pc in range(d.g)]
        return np.array([X[i] if 0 <= i < X.shape[0] else 0.0 for i in idx])
    out = []
    for pz in range(d.planes):
        for pr in range(d.m_b):
            for pc in range(d.g):
                c = [origin[-2] - radius + pr, origin[-1] - radius + pc]
                if ndim == 3:
                    c = [origin[0] - radius + pz] + c
                ok = all(0 <= c[i] < X.shape[i] for i in range(ndim))
                out.append(X[tuple(c)] if ok else 0.0)
    return np.array(out)


@pytest.mark.parametrize("ndim,k,r1,r2", [(2, 3, 8, 8), (2, 5, 4, 4), (3, 3, 8, 2), (1, 5, 16, 1),
                                          (2, 7, 16, 4)])
def test_morphed_tiles_reproduce_direct_oracle(ndim, k, r1, r2):
    # Same-size grid with a zero halo: A' . patch equals one direct sweep.
    g = synthetic.rng(23)
    r = (k - 1) // 2
    w = g.integers(-3, 4, size=(k,) * ndim).astype(np.float64)
    a, s, d = T.morph(w, r1, r2)
    dims = {1: (3 * r1,), 2: (2 * r2, 2 * r1), 3: (3, 2 * r2, r1)}[ndim]
    X = g.integers(-9, 10, size=dims).astype(np.float64)
    want = direct.run(X, w, 1)
    if ndim == 1:
        for x0 in range(0, dims[0], r1):
            out = a @ padded_patch(X, d, (x0,), r)
            assert np.array_equal(out, want[x0:x0 + r1])
    else:
        zs = range(dims[0]) if ndim == 3 else [None]
        for z in zs:
            for y0 in range(0, dims[-2], r2):
                for x0 in range(0, dims[-1], r1):
                    origin = (y0, x0) if z is None else (z, y0, x0)
                    out = (a @ padded_patch(X, d, origin, r)).reshape(r2, r1)
                    ref = want[y0:y0 + r2, x0:x0 + r1] if z is None else \
                        want[z, y0:y0 + r2, x0:x0 + r1]
                    assert np.array_equal(out, ref)


@pytest.mark.parametrize("k,r1,r2", SHAPES_2D)
def test_pit_invariance_eq5(k, r1, r2):
    g = synthetic.rng(24)
    w = g.integers(-5, 6, size=(k, k)).astype(np.float64)
    a, s, d = T.morph(w, r1, r2)
    pairs, _z = T.plane_pairs(d)
    perm = T.group(pairs, 64)
    Bp = g.integers(-7, 8, size=(d.k_prime, 5)).astype(np.float64)
    Bpp = np.zeros((len(perm), 5))
    for kk, c in enumerate(perm):
        if c != T.ZETA:
            Bpp[kk] = Bp[c]
    assert np.array_equal(T.permuted(a, perm) @ Bpp, a @ Bp)
    # the permutation is a bijection onto the real columns
    real = sorted(c for c in perm if c != T.ZETA)
    assert real == list(range(d.k_prime))
    assert len(perm) % 64 == 0


@pytest.mark.parametrize("k,r1,r2", SHAPES_2D)
def test_theorem1_pairs_conflict_free_and_groups_valid(k, r1, r2):
    a, s, d = T.morph(np.ones((k, k)), r1, r2)
    pairs, _z = T.plane_pairs(d)
    for (i, j) in pairs:
        assert not T.conflict(s, i, j)
        if j != T.ZETA:
            # Theorem 2 (i): matched columns are at least k apart in the block
            # index or in the column index of one block.
            (bi, ci), (bj, cj) = divmod(i, d.g), divmod(j, d.g)
            assert (abs(bj - bi) >= k and ci == cj) or (bi == bj and abs(cj - ci) >= k)
    perm = T.group(pairs, 64)
    for j in range(len(perm) // 4):
        cols = [c for c in perm[4 * j:4 * j + 4] if c != T.ZETA]
        assert matchers.group_ok(s, cols)


@pytest.mark.parametrize("k,r1,r2", SHAPES_2D)
def test_theorem2_zero_count(k, r1, r2):
    d = T.morph_dims(k, r1, r2, 2)
    _p, z = T.plane_pairs(d)
    assert z == T.thm2_zero_count(d)


@pytest.mark.parametrize("k,g", [(3, 3), (3, 4), (3, 5), (3, 6), (3, 7), (5, 6), (5, 9), (7, 10),
                                 (3, 10), (5, 12), (7, 14)])
def test_theorem2_local_optimality_by_exhaustive_search(k, g):
    # One local staircase (r2 = 1, one kernel row): Algorithm 1's in-block
    # matching leaves the fewest zero nodes possible.
    r1 = g - k + 1
    a, s, d = T.morph(np.ones(k), r1, 1)
    _p, z = T.plane_pairs(d)
    assert z == matchers.min_zero_pairing(s)


@pytest.mark.parametrize("k,r1,r2,alg1,pairmin", [
    (3, 1, 1, 9, 9), (3, 2, 1, 6, 6), (3, 2, 2, 4, 4), (3, 3, 1, 3, 3), (3, 4, 1, 0, 0),
    (3, 3, 2, 2, 2), (3, 5, 1, 3, 1), (3, 3, 3, 1, 1),
])
def test_alg1_against_exhaustive_pairing(k, r1, r2, alg1, pairmin):
    # Expected values: Algorithm 1 run by hand on the staircase, and the
    # exhaustive optimum (which can be smaller: Theorem 2 argues per
    # subgraph, and cross-block pairs can beat it).
    a, s, d = T.morph(np.ones((k, k)), r1, r2)
    _p, z = T.plane_pairs(d)
    assert z == alg1
    assert matchers.min_zero_pairing(s) == pairmin


def test_exact_24_can_beat_pair_relaxation():
    # k=3, (r1, r2) = (3, 2): 20 columns.  Algorithm 1 leaves 2 zero nodes,
    # which with rounding to groups of 4 means 4 pad columns, while an exact
    # 2:4 grouping needs none.
    a, s, d = T.morph(np.ones((3, 3)), 3, 2)
    pairs, z = T.plane_pairs(d)
    pads = len(T.group(pairs, 4)) - d.k_prime
    assert (z, pads) == (2, 4)
    assert matchers.min_pad_groups(s) == 0


@pytest.mark.parametrize("ndim,k,r1,r2", [(2, 3, 8, 8), (2, 7, 8, 8), (2, 13, 8, 8), (2, 13, 16, 4),
                                          (3, 3, 8, 8), (1, 5, 16, 1), (2, 5, 16, 4)])
def test_compression_is_lossless(ndim, k, r1, r2):
    g = synthetic.rng(25)
    w = g.uniform(-1, 1, size=(k,) * ndim)
    a, s, d = T.morph(w, r1, r2)
    pairs, _z = T.plane_pairs(d)
    perm = T.group(pairs, 64)
    vals, meta = T.compress(a, s, perm)
    app = T.permuted(a, perm)
    dec = np.zeros_like(app)
    for i in range(app.shape[0]):
        for j in range(len(perm) // 4):
            i0, i1 = meta[i, j]
            assert 0 <= i0 < i1 <= 3
            dec[i, 4 * j + i0] += vals[i, 2 * j]
            dec[i, 4 * j + i1] += vals[i, 2 * j + 1]
    assert np.array_equal(dec, app)


def test_compression_rejects_dense_group():
    s = np.ones((1, 4), dtype=bool)
    with pytest.raises(ValueError):
        T.compress(np.ones((1, 4)), s, [0, 1, 2, 3])


def test_gather_lut_points_at_perm_columns():
    d = T.morph_dims(3, 8, 8, 3)
    pairs, _ = T.plane_pairs(d)
    perm = T.group(pairs, 64)
    lut = T.gather_lut(d, perm)
    for kk, c in enumerate(perm):
        if c == T.ZETA:
            assert tuple(lut[kk]) == (-1, -1, -1)
        else:
            pz, pr, pc = lut[kk]
            assert (pz * d.m_b + pr) * d.g + pc == c


# ---------------------------------------------------------------- split

def test_rne_matches_numpy_binary16():
    # numpy converts float64 to float16 with a single correct rounding.
    g = synthetic.rng(26)
    xs = np.concatenate([g.uniform(-70000, 70000, 2000), g.uniform(-1, 1, 2000),
                         g.uniform(-1e-4, 1e-4, 2000), 2.0 ** g.uniform(-26, 16, 2000)])
    for x in xs:
        r = fpformat.round_rne(float(x), fpformat.BINARY16)
        with np.errstate(over="ignore"):
            n = float(np.float16(x))
        if r is None:
            assert math.isinf(n)
        else:
            assert r == n


def test_rne_matches_torch_bfloat16_on_float32_inputs():
    torch = pytest.importorskip("torch")
    g = synthetic.rng(27)
    xs = np.concatenate([g.uniform(-1, 1, 3000), 2.0 ** g.uniform(-130, 120, 3000)]).astype(np.float32)
    ref = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float32).numpy()
    for x, rv in zip(xs, ref):
        assert fpformat.round_rne(float(x), fpformat.BFLOAT16) == float(rv)


def test_rne_ties_go_to_even():
    f = fpformat.BINARY16
    assert fpformat.round_rne(1 + 2 ** -11, f) == 1.0
    assert fpformat.round_rne(1 + 3 * 2 ** -11, f) == 1 + 2 ** -9
    assert fpformat.round_rne(65519.0, f) == 65504.0
    assert fpformat.round_rne(65520.0, f) is None
    assert fpformat.round_rne(2 ** -25, f) == 0.0          # tie to even (zero)
    assert fpformat.round_rne(3 * 2 ** -25, f) == 2 ** -23  # tie to even subnormal
    b = fpformat.BFLOAT16
    assert fpformat.round_rne(1 + 2 ** -8, b) == 1.0
    assert fpformat.round_rne(1 + 3 * 2 ** -8, b) == 1 + 2 ** -6


@pytest.mark.parametrize("fmt,bound", [("f16", 2.0 ** -22), ("bf16", 2.0 ** -16)])
def test_split_reconstruction_bound(fmt, bound):
    g = synthetic.rng(28)
    vals = g.uniform(-1, 1, size=(40, 25)) * (2.0 ** g.integers(-6, 6, size=(40, 25)))
    hi, lo = T.split_hilo(vals, fmt)
    dec = fpformat.f16_value if fmt == "f16" else fpformat.bf16_value
    sigma = T.SIGMA[fmt]
    for idx in np.ndindex(*vals.shape):
        c = float(vals[idx])
        rec = dec(int(hi[idx])) + dec(int(lo[idx])) / sigma
        # lo is rounded in the format's own grid: half its smallest subnormal
        # spacing, unscaled by sigma, is the absolute floor of the error.
        floor = (2.0 ** -25 if fmt == "f16" else 2.0 ** -134) / sigma
        assert abs(c - rec) <= bound * abs(c) + floor


def test_three_part_split():
    """Three-part bfloat16 split: every part a bfloat16 number, each the
    rounding of what the parts before it leave (each at most 2^-8 of the one
    before), so |c - (hi + mid + lo)| is at most half a bfloat16 spacing of
    the last remainder (about 2^-27 |c|; asserted at 2^-26), and the sum
    reproduces c exactly when c has 24 significant bits or fewer (an FP32
    number).  Pinned by exact rational arithmetic."""
    from fractions import Fraction
    g = synthetic.rng(29)
    vals = g.uniform(-1, 1, size=(30, 20)) * (2.0 ** g.integers(-6, 6, size=(30, 20)))
    hi, mid, lo = T.split_three_bf16(vals)
    for idx in np.ndindex(*vals.shape):
        c = float(vals[idx])
        parts = [fpformat.bf16_value(int(x[idx])) for x in (hi, mid, lo)]
        assert abs(parts[1]) <= abs(parts[0]) * 2.0 ** -8 and abs(parts[2]) <= abs(parts[1]) * 2.0 ** -8
        err = abs(Fraction(c) - sum(Fraction(v) for v in parts))
        assert err <= Fraction(abs(c)) * Fraction(1, 2 ** 26)
    # FP32 numbers split exactly
    f32 = vals.astype(np.float32).astype(np.float64)
    hi, mid, lo = T.split_three_bf16(f32)
    for idx in np.ndindex(*f32.shape):
        parts = [fpformat.bf16_value(int(x[idx])) for x in (hi, mid, lo)]
        assert sum(Fraction(v) for v in parts) == Fraction(float(f32[idx]))


def test_split_overflow_raises():
    with pytest.raises(OverflowError):
        T.split_hilo(np.array([70000.0]), "f16")


# ---------------------------------------------------------------- model

def test_model_hand_computed():
    with open(os.path.join(GOLDEN, "model_box2d9p_10240.json")) as f:
        gold = json.load(f)
    t, tc, tg, ts, kpad = T.model_time(3, 2, 8, 8, (10240, 10240), elem_bytes=4, coef_bytes=2,
                                       passes=3, planes_state=1)
    assert kpad == gold["K_pad"]
    assert math.isclose(tc, gold["T_compute_s"], rel_tol=1e-12)
    assert math.isclose(tg, gold["T_global_s"], rel_tol=1e-12)
    assert math.isclose(ts, gold["T_shared_s"], rel_tol=1e-12)
    assert math.isclose(t, gold["T_s"], rel_tol=1e-12)


# ---------------------------------------------------------------- fusion

@pytest.mark.parametrize("ndim,radius,steps", [(1, 2, 2), (2, 1, 2), (2, 3, 2), (2, 1, 3), (3, 1, 2)])
def test_composed_stencil_equals_stepwise_on_periodic_grid(ndim, radius, steps):
    g = synthetic.rng(29)
    k = 2 * radius + 1
    w = g.uniform(-1, 1, size=(k,) * ndim)
    c = T.compose(w, steps)
    assert c.shape == ((steps * (k - 1) + 1),) * ndim
    dims = {1: (41,), 2: (19, 23), 3: (9, 10, 11)}[ndim]
    x = g.random(dims)
    a = direct.run(x, c, 1, periodic=True)
    b = direct.run(x, w, steps, periodic=True)
    assert np.max(np.abs(a - b)) <= 1e-13


def test_composed_sum_is_power_of_sum():
    w = synthetic.heat2d_coeffs()
    c = T.compose(w, 3)
    assert c.sum() == 1.0           # dyadic, exact
    assert c.shape == (7, 7)


# ----------------------------------------------------------------------------
# structure-aware kernel orders (beyond the paper's bounding-box structure)

def _star_w(radius, fuse, seed=45):
    w, _ = synthetic.random_coeffs("star", radius, 2, seed=seed, grid_shape=(64, 64))
    w = np.asarray(w, dtype=np.float64)
    return T.compose(w, fuse) if fuse > 1 else w


@pytest.mark.parametrize("k,r1,r2", [(3, 8, 8), (7, 8, 8), (13, 16, 2), (7, 8, 4)])
def test_compaction_is_identity_for_box_stencils(k, r1, r2):
    """A box stencil uses every patch column: both orders are the plain ones."""
    w = synthetic.random_coeffs("box", (k - 1) // 2, 2, seed=7, grid_shape=(64, 64))[0]
    a, s, d = T.morph(np.asarray(w, dtype=np.float64), r1, r2)
    perm = T.group(T.plane_pairs(d)[0], 64)
    assert T.compact_sparse_order(a, perm, 64) == perm
    natural = list(range(d.k_prime)) + [T.ZETA] * (-d.k_prime % 32)
    assert T.compact_dense_order(a, 32) == natural


@pytest.mark.parametrize("radius,fuse,r1,r2", [(3, 1, 8, 8), (3, 1, 8, 4), (3, 1, 16, 2), (3, 2, 16, 2),
                                                (3, 2, 16, 1), (3, 2, 8, 8), (2, 1, 8, 8), (1, 1, 8, 8)])
def test_compacted_orders_are_complete_and_24_valid(radius, fuse, r1, r2):
    """Brute force on A' itself: every used column appears exactly once, every
    4-group holds at most two nonzeros per row, every B register is a zero
    pair or two horizontally adjacent columns starting at an even column (the
    sparse order keeps Algorithm 1's registers, so only where those are), and
    K never grows."""
    a, s, d = T.morph(_star_w(radius, fuse), r1, r2)
    used = {c for c in range(d.k_prime) if np.any(a[:, c] != 0.0)}
    perm = T.group(T.plane_pairs(d)[0], 64)

    def registers_adjacent(order):
        for kk in range(0, len(order), 2):
            x, y = order[kk], order[kk + 1]
            if x == T.ZETA and y == T.ZETA:
                continue
            if not (x != T.ZETA and y == x + 1 and (x % d.g) % 2 == 0):
                return False
        return True

    orders = [(T.compact_sparse_order(a, perm, 64), 64, registers_adjacent(perm)),
              (T.compact_sparse_order(a, perm, 64, d.g), 64, True), (T.compact_dense_order(a, 32), 32, True)]
    for order, frag, adjacent in orders:
        assert len(order) % frag == 0
        cols = [c for c in order if c != T.ZETA]
        assert len(cols) == len(set(cols))
        assert used <= set(cols)
        if adjacent:
            assert registers_adjacent(order)
        for kk in range(0, len(order), 2):
            if order[kk] != T.ZETA or order[kk + 1] != T.ZETA:
                assert order[kk] in used or order[kk + 1] in used
    for sparse in (T.compact_sparse_order(a, perm, 64), T.compact_sparse_order(a, perm, 64, d.g)):
        assert len(sparse) <= len(perm)
        for j in range(0, len(sparse), 4):
            cols = [c for c in sparse[j:j + 4] if c != T.ZETA]
            assert np.all(np.count_nonzero(a[:, cols], axis=1) <= 2)


@pytest.mark.parametrize("k,r1,r2", [(7, 8, 4), (7, 16, 2), (7, 8, 2), (7, 16, 4), (3, 16, 2), (3, 8, 2)])
def test_aligned_repairing_of_box_layouts(k, r1, r2):
    """Box stencils at tiles where Algorithm 1 leaves in-block pairs
    (u, u + s2) with s2 odd: the aligned order takes those groups apart into
    dominoes (pc, pc + 1), pc even, and re-pairs them.  Brute force on A':
    every column once, at most two nonzeros per row in every 4-group, every
    register an aligned domino, and no more K chunks than Algorithm 1's."""
    w = synthetic.random_coeffs("box", (k - 1) // 2, 2, seed=7, grid_shape=(64, 64))[0]
    a, s, d = T.morph(np.asarray(w, dtype=np.float64), r1, r2)
    perm = T.group(T.plane_pairs(d)[0], 64)
    order = T.compact_sparse_order(a, perm, 64, d.g)
    cols = [c for c in order if c != T.ZETA]
    assert sorted(cols) == list(range(d.k_prime))
    assert len(order) <= len(perm)
    for kk in range(0, len(order), 2):
        x, y = order[kk], order[kk + 1]
        assert (x == T.ZETA and y == T.ZETA) or (y == x + 1 and (x % d.g) % 2 == 0)
    for j in range(0, len(order), 4):
        c4 = [c for c in order[j:j + 4] if c != T.ZETA]
        assert np.all(np.count_nonzero(a[:, c4], axis=1) <= 2)
    # Algorithm 1's own order is not aligned at these tiles
    assert any(not (order_x == T.ZETA or (perm[kk + 1] == order_x + 1 and (order_x % d.g) % 2 == 0))
               for kk, order_x in ((kk, perm[kk]) for kk in range(0, len(perm), 2)))


def test_compaction_counts_fused_13_point_star_at_16x2():
    """Two fused 13-point stars (radius 6, 61 points) at tile (16,2): the
    28 x 14 patch uses all 28 columns of rows 6-7 (the centre row of the
    stencil), columns 3..24 of rows 3-5 and 8-10 (|dy| <= 3 reaches |dx| <= 3)
    and columns 6..21 of rows 0-2 and 11-13 (|dy| >= 4 only at dx = 0):
    2*28 + 6*22 + 6*16 = 284 of 392 columns.  Algorithm 1 pairs block 0 with
    block 13 (8 groups used, 6 empty) and the other blocks' columns t with
    t + 14 (per row: rows 6-7 seven full groups; rows 3-5 and 8-10 five full,
    two half used; rows 1-2 and 11-12 one full, six half used), so 56 groups
    stay, 36 dominoes are re-paired and 6 groups go.  At most 36 new groups
    and at least 18: between 74 and 92 groups, and the re-pairing must keep
    it within 80 (K = 320, 5 chunks of 64 instead of 7)."""
    a, s, d = T.morph(_star_w(3, 2), 16, 2)
    used = [c for c in range(d.k_prime) if np.any(a[:, c] != 0.0)]
    assert len(used) == 284
    perm = T.group(T.plane_pairs(d)[0], 64)
    assert len(perm) == 448
    holds = lambda dom: any(c != T.ZETA and c in set(used) for c in dom)
    kinds = [(holds(perm[j:j + 2]), holds(perm[j + 2:j + 4])) for j in range(0, len(perm), 4)
             if any(c != T.ZETA for c in perm[j:j + 4])]
    assert sum(1 for u in kinds if u[0] and u[1]) == 56
    assert sum(1 for u in kinds if u[0] != u[1]) == 36
    assert sum(1 for u in kinds if not u[0] and not u[1]) == 6
    sparse = T.compact_sparse_order(a, perm, 64)
    assert len(sparse) == 320
    groups = [sparse[j:j + 4] for j in range(0, len(sparse), 4) if any(c != T.ZETA for c in sparse[j:j + 4])]
    assert 74 <= len(groups) <= 80
    assert groups[:56] == [perm[j:j + 4] for j in range(0, len(perm), 4)
                           if holds(perm[j:j + 2]) and holds(perm[j + 2:j + 4])]


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_points_box_sweep_equals_point_sum(ndim):
    """A stencil given as points: the oracle's box of it, swept by the direct
    oracle, equals sum_i c_i x~[p + o_i] written out point by point on a
    tiny zero-halo grid (brute force, no box involved)."""
    from oracle import direct
    rng = np.random.default_rng(7 + ndim)
    offs = {tuple(int(v) for v in rng.integers(-2, 3, ndim)) for _ in range(6)} | {(0,) * ndim, (2,) + (0,) * (ndim - 1)}
    offs = sorted(offs)
    c = rng.uniform(-1, 1, len(offs))
    w = T.points_box(offs, c)
    assert w.shape == (5,) * ndim and np.count_nonzero(w) == len(offs)
    shape = {1: (11,), 2: (6, 7), 3: (4, 5, 6)}[ndim]
    x = rng.uniform(0, 1, shape)
    want = np.zeros(shape)
    for p in np.ndindex(*shape):
        for o, ci in zip(offs, c):
            q = tuple(a + b for a, b in zip(p, o))
            if all(0 <= qi < n for qi, n in zip(q, shape)):
                want[p] += ci * x[q]
    got = direct.run(x, w, 1)
    assert np.allclose(got, want, rtol=0, atol=1e-14)


def test_points_box_rejects_repeats_and_sizes_radius():
    assert T.points_box([(0, 0)], [2.0]).shape == (3, 3)
    assert T.points_box([(0, 3)], [1.0]).shape == (7, 7)
    with pytest.raises(ValueError):
        T.points_box([(0, 1), (0, 1)], [1.0, 2.0])
