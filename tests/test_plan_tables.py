"""Plan tables of libsparstencil (host-only plans, no GPU) against the oracle's
independent re-derivation: permutation, compressed values, metadata, hi/lo
parts and gather LUT must match bit for bit; the layout-exploration model must
give the same times and the same argmin (Section 3.3, Eqs. 6-11)."""
import numpy as np
import pytest

import synthetic
from oracle import tables as T

native = pytest.importorskip("paper_2506_22969_amd.native")


def host_plan(shape, radius, w, dims, dtype="f32_split_f16", **kw):
    return native.Plan(shape, radius, w, dims, dtype, host_only=True, engine="smfmac", **kw)


CASES = [
    ("box", 1, 2, (10240, 10240), 8, 8),
    ("box", 1, 2, (10240, 10240), 16, 4),
    ("star", 1, 2, (4096, 4096), 8, 8),
    ("box", 1, 2, (300, 257), 0, 0),
    ("box", 1, 3, (512, 512, 512), 8, 4),
    ("star", 1, 3, (64, 96, 128), 0, 0),
]


@pytest.mark.parametrize("shape,radius,ndim,dims,r1,r2", CASES)
@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_tables_bit_exact(shape, radius, ndim, dims, r1, r2, fmt):
    w, _ = synthetic.random_coeffs(shape, radius, ndim, seed=5, grid_shape=dims)
    dtype = "f32_split_f16" if fmt == "f16" else "f32_split_bf16"
    with host_plan(shape, radius, w, dims, dtype, r1=r1, r2=r2) as p:
        info = p.info
        assert info["engine_name"] == "smfmac"
        a, s, d = T.morph(T.bounding_box(shape, radius, ndim, w), info["r1"], info["r2"])
        assert (info["m_prime"], info["k_prime"]) == (d.m_prime, d.k_prime)
        pairs, zeros = T.plane_pairs(d)
        perm = T.group(pairs, 64)
        assert info["zeros"] == zeros
        assert info["k_pad"] == len(perm)
        assert np.array_equal(p.table(native.Q_PERM), np.array(perm, dtype=np.int32))
        vals, meta = T.compress(a, s, perm)
        assert np.array_equal(p.table(native.Q_VALUES), vals.reshape(-1))
        assert np.array_equal(p.table(native.Q_META), meta.reshape(-1).astype(np.uint8))
        hi, lo = T.split_hilo(vals, fmt)
        assert np.array_equal(p.table(native.Q_HI), hi.reshape(-1))
        assert np.array_equal(p.table(native.Q_LO), lo.reshape(-1))
        lut = T.gather_lut(d, perm)
        assert np.array_equal(p.table(native.Q_LUT), lut.reshape(-1).astype(np.int32))


@pytest.mark.parametrize("dims", [(10240, 10240), (1024, 1024), (64, 200)])
def test_model_and_argmin_match_oracle(dims):
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=5, grid_shape=dims)
    with host_plan("box", 1, w, dims) as p:
        rows = p.table(native.Q_MODEL).reshape(-1, 7)
        info = p.info
    cands = [(int(r[0]), int(r[1])) for r in rows]
    best, table = T.explore(3, 2, dims, cands, elem_bytes=4, coef_bytes=2, passes=3, planes_state=1)
    for r in rows:
        t, tc, tg, ts, kpad = table[(int(r[0]), int(r[1]))]
        assert r[2] == pytest.approx(t, rel=1e-12)
        assert r[3] == pytest.approx(tc, rel=1e-12)
        assert r[4] == pytest.approx(tg, rel=1e-12)
        assert r[5] == pytest.approx(ts, rel=1e-12)
        assert int(r[6]) == kpad
    assert (info["r1"], info["r2"]) == best


def test_heat2d_coefficients_split_exactly():
    # 0.5 and 0.125 are binary16 numbers: every lo part is zero.
    w = synthetic.heat2d_coeffs()
    with host_plan("star", 1, w, (256, 256)) as p:
        assert np.all(p.table(native.Q_LO) == 0)


def test_fused_plan_uses_composed_coefficients():
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=5)
    with native.Plan("box", 1, w, (512, 512), "f32", boundary="periodic", fuse_steps=2,
                     engine="direct", host_only=True) as p:
        c = p.table(native.Q_COEFFS).reshape(5, 5)
        assert p.info["k"] == 5
    assert np.array_equal(c, T.compose(w, 2))


def test_invalid_arguments():
    w = synthetic.heat2d_coeffs()
    with pytest.raises(native.SparStencilError):
        native.Plan("star", 1, np.ones((3, 3)), (64, 64), "f32_split_f16", host_only=True)  # star off-axis
    with pytest.raises(native.SparStencilError):
        native.Plan("box", 1, w, (0, 64), "f32_split_f16", host_only=True)
    with pytest.raises(native.SparStencilError):
        native.Plan("box", 1, w, (64, 64), "f32", fuse_steps=2, host_only=True)  # fusion needs periodic
    big = w * 1e6
    with pytest.raises(native.SparStencilError):
        native.Plan("box", 1, big, (64, 64), "f32_split_f16", engine="smfmac", host_only=True)


@pytest.mark.parametrize("shape,seed", [("star", 45), ("box", 277)])
@pytest.mark.parametrize("fuse", [1, 2])
def test_radius3_planes_tables_and_model(shape, seed, fuse):
    # Star-2D13P / Box-2D49P on bfloat16 hi+lo planes, unfused (k = 7) and
    # with two fused sweeps (k = 13): the kernel's tables against the oracle's
    # re-derivation from the (composed) coefficients, and the tile the model
    # picks among the instantiated ones.
    dims = (8192, 8192)
    w, _ = synthetic.random_coeffs(shape, 3, 2, seed=seed, grid_shape=dims)
    with native.Plan(shape, 3, w, dims, "split_bf16", boundary="periodic", fuse_steps=fuse,
                     engine="smfmac", host_only=True) as p:
        info = p.info
        wc = p.table(native.Q_COEFFS)
        rows = p.table(native.Q_MODEL).reshape(-1, 7)
        wf = T.compose(w, fuse) if fuse > 1 else w
        k = 7 if fuse == 1 else 13
        assert info["k"] == k
        assert np.array_equal(wc, wf.reshape(-1))
        a, s, d = T.morph(T.bounding_box("box", (k - 1) // 2, 2, wf), info["r1"], info["r2"])
        pairs, zeros = T.plane_pairs(d)
        perm = T.group(pairs, 64)
        assert info["k_pad"] == len(perm) and info["zeros"] == zeros
        assert np.array_equal(p.table(native.Q_PERM), np.array(perm, dtype=np.int32))
        vals, meta = T.compress(a, s, perm)
        assert np.array_equal(p.table(native.Q_VALUES), vals.reshape(-1))
        assert np.array_equal(p.table(native.Q_META), meta.reshape(-1).astype(np.uint8))
        hi, lo = T.split_hilo(vals, "bf16")
        assert np.array_equal(p.table(native.Q_HI), hi.reshape(-1))
        assert np.array_equal(p.table(native.Q_LO), lo.reshape(-1))
    cands = [(int(r[0]), int(r[1])) for r in rows]
    best, table = T.explore(k, 2, dims, cands, elem_bytes=2, coef_bytes=2, passes=3, planes_state=2)
    for r in rows:
        t = table[(int(r[0]), int(r[1]))][0]
        assert r[2] == pytest.approx(t, rel=1e-12)
    assert (info["r1"], info["r2"]) == best


def test_planes_rows_must_be_a_multiple_of_8_for_mma():
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=(64, 64))
    with pytest.raises(native.SparStencilError):
        native.Plan("box", 1, w, (64, 60), "split_bf16", engine="smfmac", host_only=True)
    with native.Plan("box", 1, w, (64, 60), "split_bf16", host_only=True) as p:
        assert p.info["engine_name"] == "direct"


def test_rows_beyond_32bit_item_offsets_fall_back_to_direct():
    """A 2-D work item of 32 rows (or a 3-D plane) must span < 2^31 bytes for
    the slab kernels; wider grids plan onto the direct engine."""
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=(64, 64))
    wide = (4, 1 << 24)                      # 32 rows x 2^24 x 4 bytes = 2^31
    with pytest.raises(native.SparStencilError):
        native.Plan("box", 1, w, wide, "f32_split_f16", engine="smfmac", host_only=True)
    with native.Plan("box", 1, w, wide, "f32_split_f16", host_only=True) as p:
        assert p.info["engine_name"] == "direct"
    with native.Plan("box", 1, w, (4, (1 << 24) - 8), "f32_split_f16", engine="smfmac", host_only=True) as p:
        assert p.info["engine_name"] == "smfmac"
    w3, _ = synthetic.random_coeffs("box", 1, 3, seed=1)
    with pytest.raises(native.SparStencilError):
        native.Plan("box", 1, w3, (3, 1 << 14, 1 << 15), "f32_split_f16", engine="smfmac", host_only=True)


@pytest.mark.parametrize("shape,radius,fuse,dtype,engine", [
    ("star", 3, 2, "split_bf16", "smfmac"), ("star", 3, 2, "split_bf16", "mfma"),
    ("star", 3, 1, "split_bf16", "smfmac"), ("star", 3, 1, "f32_split_f16", "mfma"),
    ("star", 3, 1, "f32_split_bf16", "smfmac"), ("star", 1, 1, "f32_split_f16", "smfmac"),
    ("box", 3, 2, "split_bf16", "smfmac"), ("box", 1, 1, "f32_split_f16", "mfma")])
def test_kernel_order_matches_oracle(shape, radius, fuse, dtype, engine):
    """The launched kernel's K order (Algorithm 1's groups compacted to the
    used columns, or the used column pairs in natural order) equals the
    oracle's, bit for bit."""
    dims = (256, 256)
    w, _ = synthetic.random_coeffs(shape, radius, 2, seed=45 if radius == 3 else 1, grid_shape=dims)
    kw = dict(boundary="periodic", fuse_steps=fuse) if fuse > 1 else {}
    if shape == "star" and radius == 3:
        # a tile on which dropping the unused columns shortens K
        kw.update(r1=8, r2=4 if engine == "smfmac" or fuse == 1 else 2)
    with native.Plan(shape, radius, w, dims, dtype, engine=engine, host_only=True, **kw) as p:
        info = p.info
        got = p.table(native.Q_KERNEL_PERM)
        wk = p.table(native.Q_COEFFS).reshape(info["k"], info["k"])
    a, s, d = T.morph(wk, info["r1"], info["r2"])
    if engine == "smfmac":
        perm = T.group(T.plane_pairs(d)[0], 64)
        _check_sparse_kernel_order(a, d, perm, got)
        ref = T.compact_sparse_order(a, perm, 64, d.g)
    else:
        ref = T.compact_dense_order(a, 32)
        assert np.array_equal(got, np.array(ref, dtype=np.int32))
    if shape == "star" and radius == 3:
        assert len(got) < (len(T.group(T.plane_pairs(d)[0], 64)) if engine == "smfmac" else -(-d.k_prime // 32) * 32)
        assert len(got) <= len(ref)


def _check_sparse_kernel_order(a, d, perm, got):
    """The sparse kernel order against the oracle: Algorithm 1's kept groups
    first, bit for bit; then the re-paired dominoes, each group two
    compatible aligned dominoes (or one and a zero domino), every used
    column exactly once, and as few groups as a maximum matching of the
    dominoes' compatibility graph gives (networkx, not the planner's
    matcher)."""
    kept, best = T.max_repairing_groups(a, perm, d.g)
    got = [int(c) for c in got]
    nk = 4 * len(kept)
    assert got[:nk] == [c for grp in kept for c in grp]
    groups = [tuple(got[j:j + 4]) for j in range(nk, len(got), 4) if any(c != T.ZETA for c in got[j:j + 4])]
    assert len(groups) == best
    for c0, c1, c2, c3 in groups:
        assert c1 == c0 + 1 and (c0 % d.g) % 2 == 0
        assert (c2 == T.ZETA and c3 == T.ZETA) or (c3 == c2 + 1 and (c2 % d.g) % 2 == 0)
        assert T.dominoes_compatible(a, (c0, c1), (c2, c3))
    used = set(int(c) for c in np.flatnonzero(T.used_columns(a)))
    cols = [c for c in got if c != T.ZETA]
    assert len(cols) == len(set(cols)) and used <= set(cols)
    for j in range(0, len(got), 4):
        c4 = [c for c in got[j:j + 4] if c != T.ZETA]
        assert np.all(np.count_nonzero(a[:, c4], axis=1) <= 2)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("r1,r2", [(8, 8), (8, 4), (16, 2), (8, 2)])
def test_repairing_is_a_maximum_matching(seed, r1, r2):
    """Radius-3 stencils with random zero patterns (about half the box):
    the sparse kernel order re-pairs the set-aside dominoes by a maximum
    matching (the paper's general matcher, Section 3.2), checked against
    networkx on the same graph; completeness and 2:4 validity by brute
    force on A'."""
    rng = np.random.default_rng(100 + seed)
    w = rng.uniform(-1, 1, (7, 7))
    w[rng.random((7, 7)) < 0.5] = 0.0
    w[3, 3] = 1.0
    dims = (64, 64)
    with native.Plan("box", 3, w, dims, "f32_split_f16", engine="smfmac", r1=r1, r2=r2, host_only=True) as p:
        got = p.table(native.Q_KERNEL_PERM)
    a, s, d = T.morph(w, r1, r2)
    _check_sparse_kernel_order(a, d, T.group(T.plane_pairs(d)[0], 64), got)


def test_zero_halo_fusion_scope():
    """Fused sweeps with a zero halo: FP32-state plans only; 2-D S = 2 (any
    radius) or S = 3 (radius 1), the band along the edges recomputed inside
    the sweep launch by the matrix kernels and by a second launch on the
    direct engine; 3-D S = 2 of radius 1, the band inside the launch; planes,
    S = 4, 2-D S = 3 beyond radius 1 and 3-D beyond S = 2 or radius 1 stay
    unsupported."""
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=(64, 64))
    with native.Plan("box", 1, w, (64, 64), "f32_split_bf16", fuse_steps=2, host_only=True) as p:
        info = p.info
        assert info["fuse_steps"] == 2 and info["k"] == 5 and info["launches_per_sweep"] == 1
    with native.Plan("box", 1, w, (64, 64), "f32_split_f16", fuse_steps=3, host_only=True) as p:
        assert p.info["k"] == 7 and p.info["launches_per_sweep"] == 1
    with native.Plan("box", 1, w, (64, 64), "f32_split_f16", fuse_steps=3, engine="direct", host_only=True) as p:
        assert p.info["k"] == 7 and p.info["launches_per_sweep"] == 2
    w3r, _ = synthetic.random_coeffs("box", 3, 2, seed=1, grid_shape=(64, 64))
    for rad, wr, dtype, fuse in [(1, w, "split_bf16", 2), (1, w, "f32_split_f16", 4), (3, w3r, "f32_split_f16", 3)]:
        with pytest.raises(native.SparStencilError):
            native.Plan("box", rad, wr, (64, 64), dtype, fuse_steps=fuse, host_only=True)
    # 3-D: two radius-1 sweeps, the band inside the launch on every engine
    w3, _ = synthetic.random_coeffs("box", 1, 3, seed=1)
    for engine in ("smfmac", "mfma", "direct"):
        with native.Plan("box", 1, w3, (8, 8, 8), "f32_split_f16", fuse_steps=2, engine=engine, host_only=True) as p:
            assert p.info["k"] == 5 and p.info["launches_per_sweep"] == 1
    for fuse, dtype in [(3, "f32_split_f16"), (2, "split_bf16")]:
        with pytest.raises(native.SparStencilError):
            native.Plan("box", 1, w3, (8, 8, 8), dtype, fuse_steps=fuse, host_only=True)
    w3r2, _ = synthetic.random_coeffs("box", 2, 3, seed=1)
    with pytest.raises(native.SparStencilError):
        native.Plan("box", 2, w3r2, (8, 8, 8), "f32_split_f16", fuse_steps=2, host_only=True)


@pytest.mark.parametrize("shape,fuse,engine,k_pad", [
    ("box", 2, "smfmac", 640), ("star", 2, "smfmac", 320), ("box", 2, "mfma", 480), ("star", 2, "mfma", 320),
    ("star", 1, "smfmac", 192), ("box", 1, "smfmac", 192), ("star", 1, "mfma", 192)])
def test_3d_kernel_order_is_the_union_order(shape, fuse, engine, k_pad):
    """3-D kernel K order: one 2-D order for every plane (the kernel gathers
    an input plane once for all plane offsets), compacted to the union of
    the columns the planes of A' use -- the oracle's compaction of the
    summed |A'| planes (sparse: Algorithm 1's groups re-paired, checked as
    the 2-D orders are; dense: the used column pairs), each plane a valid
    2:4 layout of its own block."""
    w, _ = synthetic.random_coeffs(shape, 1, 3, seed=29 if shape == "star" else 70)
    kw = dict(fuse_steps=fuse) if fuse > 1 else {}
    with native.Plan(shape, 1, w, (40, 48, 264), "f32_split_f16", engine=engine, host_only=True, **kw) as p:
        info = p.info
        got = p.table(native.Q_KERNEL_PERM)
        wk = p.table(native.Q_COEFFS).reshape((info["k"],) * 3)
    k = info["k"]
    assert len(got) == k_pad
    planes = [T.morph(wk[pz], info["r1"], info["r2"]) for pz in range(k)]
    d = planes[0][2]
    plane = d.m_b * d.g
    union = sum(np.abs(a) for a, _, _ in planes)
    one = got[:len(got) // k]
    for pz in range(k):
        blk = got[pz * len(one):(pz + 1) * len(one)]
        assert np.array_equal(blk, np.where(one >= 0, one + pz * plane, one))
        a = planes[pz][0]
        for j in range(0, len(one), 4):
            cols = [int(c) for c in one[j:j + 4] if c >= 0]
            if engine == "smfmac":
                assert np.all(np.count_nonzero(a[:, cols], axis=1) <= 2)
    if engine == "smfmac":
        _check_sparse_kernel_order(union, d, T.group(T.plane_pairs(d)[0], 64), one)
    else:
        assert np.array_equal(one, np.array(T.compact_dense_order(union, 32), dtype=np.int32))


@pytest.mark.parametrize("radius,fuse", [(1, 1), (2, 1), (1, 3), (2, 3), (4, 2), (8, 1)])
@pytest.mark.parametrize("engine", ["smfmac", "mfma"])
def test_1d_kernel_order_is_a_valid_layout(radius, fuse, engine):
    """The 1-D kernels' K order (one chunk) holds every column of the
    oracle's A' (16 x (15 + k)) once, pairs horizontally adjacent columns in
    each B register, and (sparse) leaves at most two nonzeros of any A' row
    in every 4-group."""
    from oracle import tables as T
    n = 5000
    w, _ = synthetic.random_coeffs("box", radius, 1, seed=3, grid_shape=(4096,))
    kw = dict(boundary="periodic", fuse_steps=fuse) if fuse > 1 else {}
    with native.Plan("box", radius, w, (n,), "f32_split_f16", engine=engine, host_only=True, **kw) as p:
        info = p.info
        order = p.table(native.Q_KERNEL_PERM)
        wk = p.table(native.Q_COEFFS)
    assert info["engine_name"] == engine and (info["r1"], info["r2"]) == (16, 1)
    assert info["k"] == 2 * radius * fuse + 1
    a, s, d = T.morph(wk.reshape(info["k"]), 16, 1)
    assert a.shape == (16, 15 + info["k"])
    assert len(order) == (64 if engine == "smfmac" else 32)
    used = sorted(int(c) for c in order if c >= 0)
    assert used == list(range(a.shape[1]))
    for v in range(0, len(order), 2):
        c0, c1 = int(order[v]), int(order[v + 1])
        assert (c0 < 0 and c1 < 0) or (c0 >= 0 and c1 == c0 + 1)
    if engine == "smfmac":
        for gq in range(0, len(order), 4):
            cols = [int(c) for c in order[gq:gq + 4] if c >= 0]
            assert np.all(np.count_nonzero(a[:, cols], axis=1) <= 2)


def test_1d_zero_halo_fusion_scope():
    """1-D zero-halo fusion: any S with r*S <= 8 (the staged halo), the two
    end bands recomputed by one more workgroup of the sweep's launch (matrix
    and direct kernels alike); beyond that it is rejected."""
    w1, _ = synthetic.random_coeffs("box", 1, 1, seed=3, grid_shape=(4096,))
    w3, _ = synthetic.random_coeffs("box", 3, 1, seed=3, grid_shape=(4096,))
    with native.Plan("box", 1, w1, (1000,), "f32_split_f16", fuse_steps=8, host_only=True) as p:
        assert p.info["launches_per_sweep"] == 1 and p.info["k"] == 17
    with native.Plan("box", 1, w1, (1000,), "f32_split_f16", fuse_steps=3, engine="direct", host_only=True) as p:
        assert p.info["launches_per_sweep"] == 1 and p.info["engine_name"] == "direct"
    with pytest.raises(native.SparStencilError):
        native.Plan("box", 3, w3, (1000,), "f32_split_f16", fuse_steps=3, host_only=True)
    with native.Plan("box", 3, w3, (1000,), "f32_split_bf16", host_only=True) as p:
        assert p.info["engine_name"] == "smfmac" and p.info["launches_per_sweep"] == 1


def test_direct_engine_refuses_radii_beyond_its_kernels():
    """The direct kernels go up to radius 6; a wider plan on that engine is
    refused when it is made, not when it runs."""
    w7 = np.zeros((15, 15))
    w7[7, :] = 1.0 / 15
    with pytest.raises(native.SparStencilError):
        native.Plan("box", 7, w7, (100, 100), "f32", engine="direct", host_only=True)
    w6 = np.zeros((13, 13))
    w6[6, :] = 1.0 / 13
    with native.Plan("box", 6, w6, (100, 100), "f32", engine="direct", host_only=True) as p:
        assert p.info["engine_name"] == "direct"


@pytest.mark.parametrize("shape,seed,fuse", [("star", 45, 2), ("box", 277, 2), ("box", 3, 1)])
def test_three_part_planes_tables(shape, seed, fuse):
    """bfloat16 hi/mid/lo planes state: the canonical tables as for two
    parts, the coefficients' hi, mid and lo parts bit-exact against the
    oracle's three-part split, and the model with six products and three
    planes."""
    dims = (8192, 8192)
    w, _ = synthetic.random_coeffs(shape, 3, 2, seed=seed, grid_shape=dims)
    with native.Plan(shape, 3, w, dims, "split3_bf16", boundary="periodic", fuse_steps=fuse,
                     engine="smfmac", host_only=True) as p:
        info = p.info
        assert info["passes"] == 6
        wf = T.compose(w, fuse) if fuse > 1 else w
        k = 7 if fuse == 1 else 13
        a, s, d = T.morph(T.bounding_box("box", (k - 1) // 2, 2, wf), info["r1"], info["r2"])
        perm = T.group(T.plane_pairs(d)[0], 64)
        assert np.array_equal(p.table(native.Q_PERM), np.array(perm, dtype=np.int32))
        vals, meta = T.compress(a, s, perm)
        hi, mid, lo = T.split_three_bf16(vals)
        assert np.array_equal(p.table(native.Q_HI), hi.reshape(-1))
        assert np.array_equal(p.table(native.Q_MID), mid.reshape(-1))
        assert np.array_equal(p.table(native.Q_LO), lo.reshape(-1))
        rows = p.table(native.Q_MODEL).reshape(-1, 7)
    cands = [(int(r[0]), int(r[1])) for r in rows]
    best, table = T.explore(k, 2, dims, cands, elem_bytes=2, coef_bytes=2, passes=6, planes_state=3)
    for r in rows:
        assert r[2] == pytest.approx(table[(int(r[0]), int(r[1]))][0], rel=1e-12)
    assert (info["r1"], info["r2"]) == best


def test_three_part_planes_scope():
    # matrix engines only, 2-D, rows a multiple of 8 values
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=(64, 64))
    for kw in (dict(engine="direct"), dict(dims=(64, 60))):
        dims = kw.pop("dims", (64, 64))
        with pytest.raises(native.SparStencilError):
            native.Plan("box", 1, w, dims, "split3_bf16", host_only=True, **kw)


def test_custom_points_plan_equals_box_plan():
    """sparstencil_plan_points builds the plan of the box holding the
    points' coefficients (the oracle's points_box), shape SS_SHAPE_CUSTOM:
    same coefficients, same kernel K order; a radius-2 point list gives a
    5-wide box; repeated offsets, offsets beyond 16 and mismatched lengths
    are rejected."""
    offs = [(0, 0), (0, -1), (-1, 0), (-1, -1), (0, -2), (2, 1)]
    c = [0.5, 0.2, 0.15, 0.1, 0.04, 0.01]
    w = T.points_box(offs, c)
    dims = (256, 256)
    with native.Plan("custom", 0, c, dims, "f32_split_f16", offsets=offs, host_only=True) as p:
        info = p.info
        wk = p.table(native.Q_COEFFS)
        perm = p.table(native.Q_KERNEL_PERM)
    with native.Plan("custom", 2, w, dims, "f32_split_f16", host_only=True) as q:
        assert np.array_equal(q.table(native.Q_KERNEL_PERM), perm)
    assert info["k"] == 5 and np.array_equal(wk.reshape(5, 5), w)
    # fewer used columns than the box: the K order drops the rest
    with native.Plan("box", 2, np.ones((5, 5)), dims, "f32_split_f16", host_only=True) as b:
        assert len(perm) <= len(b.table(native.Q_KERNEL_PERM))
    for bad_offs, bad_c in [([(0, 1), (0, 1)], [1.0, 2.0]), ([(0, 17)], [1.0]), ([(0, 1)], [1.0, 2.0])]:
        with pytest.raises((native.SparStencilError, ValueError)):
            native.Plan("custom", 0, bad_c, dims, "f32_split_f16", offsets=bad_offs, host_only=True)
    # a custom box pattern is not held to the star rule
    with native.Plan("custom", 1, np.arange(9.0).reshape(3, 3), dims, "f32_split_f16", host_only=True) as p:
        assert p.info["k"] == 3
