"""GPU parity: libsparstencil's HIP engines against the FP64 oracle, through
the C ABI, on seeded synthetic grids.

Tolerances (normwise relative error after T sweeps): each split-precision
sweep is bounded by split_step_bound(fmt, n_mma) * sum|c| relative to the
largest state value; the tests allow T times that bound.  The direct FP32
engine gets T * (P + 1) * 2^-24 * sum|c|, FP64 1e-13.  Binary16-split and
FP32 results are also held to the stated bounds (STATED_F32 = 1e-5, and
STATED_SPLIT = 1e-6 for the fused workloads that reach it), which on the
100-sweep workloads sit a few times above the measured errors.
"""
import numpy as np
import pytest

import synthetic
from oracle import direct as oracle_direct

from .helpers import (STATED_F32, STATED_SPLIT, apriori_bound, cone_sample, normwise_err, sample_points,
                      split_step_bound)

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_2506_22969_amd.native")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def stream():
    return torch.cuda.current_stream().cuda_stream


def run_plan(plan, x0: np.ndarray, steps: int) -> np.ndarray:
    a = torch.from_numpy(np.ascontiguousarray(x0)).to(DEV)
    b = torch.empty_like(a)
    plan.run(a, b, steps, stream())
    torch.cuda.synchronize()
    return b.cpu().numpy()


def n_mma_of(info) -> int:
    # MMAs accumulating into one output: 3 passes per 64-wide (sparse) or
    # 32-wide (dense) K chunk
    chunk = 64 if info["engine_name"] == "smfmac" else 32
    return 3 * info["k_pad"] // chunk


def tol_for(info, w, steps, dtype):
    s = float(np.abs(w).sum())
    if info["engine_name"] == "direct":
        p = np.count_nonzero(w)
        return steps * (p + 1) * 2.0 ** -24 * s * 2
    fmt = "f16" if dtype == "f32_split_f16" else "bf16"
    return steps * split_step_bound(fmt, n_mma_of(info)) * s


SMALL = [(200, 300), (64, 128), (129, 131), (7, 5), (1, 200), (300, 1), (256, 256)]


@pytest.mark.parametrize("engine", ["smfmac", "mfma", "direct"])
@pytest.mark.parametrize("dims", SMALL)
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_box9_f16_split_small(engine, dims, boundary):
    w, seed = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=dims)
    x0 = synthetic.grid_f32(dims, seed=0)
    steps = 5
    with native.Plan("box", 1, w, dims, "f32_split_f16", boundary=boundary, engine=engine) as p:
        info = p.info
        assert info["engine_name"] == engine
        got = run_plan(p, x0, steps)
    ref = oracle_direct.run(x0.astype(np.float64), w, steps, periodic=(boundary == "periodic"))
    err = normwise_err(got, ref)
    tol = tol_for(info, w, steps, "f32_split_f16")
    print(f"engine={engine} dims={dims} bc={boundary} err={err:.3e} tol={tol:.3e}")
    assert err <= tol
    assert err <= STATED_F32


@pytest.mark.parametrize("engine", ["smfmac", "mfma"])
@pytest.mark.parametrize("r1,r2", [(8, 8), (16, 4)])
def test_bf16_split_and_tiles(engine, r1, r2):
    dims = (333, 517)
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=3, grid_shape=dims)
    x0 = synthetic.grid_f32(dims, seed=4)
    steps = 6
    for dtype in ("f32_split_f16", "f32_split_bf16"):
        with native.Plan("box", 1, w, dims, dtype, engine=engine, r1=r1, r2=r2) as p:
            info = p.info
            assert (info["r1"], info["r2"]) == (r1, r2)
            got = run_plan(p, x0, steps)
        ref = oracle_direct.run(x0.astype(np.float64), w, steps)
        err = normwise_err(got, ref)
        tol = tol_for(info, w, steps, dtype)
        print(f"{engine} ({r1},{r2}) {dtype} err={err:.3e} tol={tol:.3e}")
        assert err <= tol


def test_star5_heat2d_f64_direct_c1():
    # Heat-2D Jacobi, 256x256 FP64, zero halo, 10 sweeps: one launch (ten
    # sweeps in LDS), equal to the oracle (every product is exact)
    w = synthetic.heat2d_coeffs()
    x0 = synthetic.grid_f64((256, 256), seed=0)
    with native.Plan("star", 1, w, (256, 256), "f64") as p:
        assert p.info["engine_name"] == "direct" and p.launch_count(10) == 1
        got = run_plan(p, x0, 10)
    ref = oracle_direct.run(x0, w, 10)
    assert normwise_err(got, ref) <= 1e-13
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("radius", [1, 2, 4])
@pytest.mark.parametrize("dims,boundary", [((256, 256), "zero"), ((129, 131), "periodic"), ((7, 5), "zero"),
                                           ((5, 9), "periodic"), ((300, 520), "zero")])
@pytest.mark.parametrize("steps", [1, 3, 16, 37])
def test_f64_temporal_blocks_equal_single_sweeps(radius, dims, boundary, steps):
    """Small FP64 grids run up to 16/r sweeps per launch in LDS: the result
    equals, bit for bit, the same sweeps run one per launch
    (sparstencil_sweep), and the FP64 oracle to 1e-13."""
    w, _ = synthetic.random_coeffs("box", radius, 2, seed=2, grid_shape=dims)
    x0 = synthetic.grid_f64(dims, seed=4)
    if boundary == "periodic" and min(dims) < radius:
        pytest.skip("periodic grid narrower than the stencil")
    with native.Plan("box", radius, w, dims, "f64", boundary=boundary, engine="direct") as p:
        assert p.launch_count(steps) == -(-steps // (16 // radius))
        got = run_plan(p, x0, steps)
        a = torch.from_numpy(x0).to(DEV)
        b = torch.empty_like(a)
        for _ in range(steps):
            p.sweep(a, b, stream())
            a, b = b, a
        torch.cuda.synchronize()
        single = a.cpu().numpy()
    assert np.array_equal(got, single)
    ref = oracle_direct.run(x0, w, steps, periodic=(boundary == "periodic"))
    assert normwise_err(got, ref) <= 1e-13


@pytest.mark.parametrize("dims", [(256, 256), (129, 131), (7, 5), (300, 520)])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_f64_mfma_engine(dims, boundary):
    # FP64 staircase product on v_mfma_f64_16x16x4: Heat-2D and a random
    # 9-point box, 10 sweeps, against the oracle at the FP64 bound
    x0 = synthetic.grid_f64(dims, seed=2)
    for shape, w in [("star", synthetic.heat2d_coeffs()),
                     ("box", synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=dims)[0])]:
        with native.Plan(shape, 1, w, dims, "f64", boundary=boundary, engine="mfma") as p:
            assert p.info["engine_name"] == "mfma"
            got = run_plan(p, x0, 10)
        ref = oracle_direct.run(x0, w, 10, periodic=(boundary == "periodic"))
        err = normwise_err(got, ref)
        print(f"f64 mfma {shape} {dims} {boundary} err={err:.3e}")
        assert err <= 1e-13


@pytest.mark.parametrize("engine", ["smfmac", "mfma", "direct"])
def test_constant_field_bit_exact(engine):
    # Heat-2D coefficients and the state 0.75 are binary16 numbers; every
    # product and partial sum is exact, so interior points equal (sum c)^T k.
    w = synthetic.heat2d_coeffs()
    dims = (96, 160)
    x0 = np.full(dims, 0.75, dtype=np.float32)
    steps = 3
    with native.Plan("star", 1, w, dims, "f32_split_f16", engine=engine) as p:
        got = run_plan(p, x0, steps)
    assert np.all(got[steps:-steps, steps:-steps] == 0.75)
    with native.Plan("star", 1, w, dims, "f32_split_f16", engine=engine, boundary="periodic") as p:
        got = run_plan(p, x0, steps)
    assert np.all(got == 0.75)


@pytest.mark.parametrize("engine", ["smfmac", "mfma"])
def test_laplacian_of_quadratic_bit_exact(engine):
    # 5-point Laplacian of a x^2 + b xy + c y^2 + d x + e y + h is 2a + 2c at
    # interior points; integer inputs below 2048 are exact binary16 values.
    lap = np.array([[0, 1, 0], [1, -4, 1], [0, 1, 0]], dtype=np.float64)
    ny, nx = 40, 44
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    a, b, c, d, e, h = 1, -1, 1, 2, -3, 5
    f = a * x * x + b * x * y + c * y * y + d * x + e * y + h
    assert np.abs(f).max() < 2048
    with native.Plan("star", 1, lap, (ny, nx), "f32_split_f16", engine=engine) as p:
        got = run_plan(p, f.astype(np.float32), 1)
    assert np.all(got[1:-1, 1:-1] == 2 * a + 2 * c)


def test_steps_zero_one_two_and_determinism():
    dims = (100, 140)
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=dims)
    x0 = synthetic.grid_f32(dims, seed=7)
    with native.Plan("box", 1, w, dims, "f32_split_f16") as p:
        assert np.array_equal(run_plan(p, x0, 0), x0)
        one = run_plan(p, x0, 1)
        two = run_plan(p, x0, 2)
        again = run_plan(p, x0, 2)
        assert p.launch_count(2) == 2
    assert np.array_equal(two, again)
    # two sweeps equal one sweep applied twice, bit for bit
    with native.Plan("box", 1, w, dims, "f32_split_f16") as p:
        twice = run_plan(p, one, 1)
    assert np.array_equal(two, twice)


def test_run_rejects_aliasing():
    dims = (64, 64)
    w = synthetic.heat2d_coeffs()
    with native.Plan("star", 1, w, dims, "f32_split_f16") as p:
        a = torch.zeros(dims, device=DEV)
        with pytest.raises(native.SparStencilError):
            p.run(a, a, 1, stream())


def test_box9_full_size_sampled():
    # The benchmark's workload: Box-2D9P on 10240^2, FP32 state, binary16
    # split on the sparse engine, 100 sweeps, zero halo; checked at sampled
    # points through their dependency cones.
    dims = (10240, 10240)
    steps = 100
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=dims)
    x0 = synthetic.grid_f32(dims, seed=0)
    with native.Plan("box", 1, w, dims, "f32_split_f16") as p:
        info = p.info
        assert info["engine_name"] == "smfmac"
        got = run_plan(p, x0, steps)
    pts = sample_points(*dims, 24, seed=1)
    ref = cone_sample(x0, w, steps, pts)
    vals = np.array([got[y, x] for (y, x) in pts], dtype=np.float64)
    err = float(np.abs(vals - ref).max() / np.abs(ref).max())
    tol = tol_for(info, w, steps, "f32_split_f16")
    print(f"full-size sampled err={err:.3e} tol={tol:.3e}")
    assert err <= tol
    # stated bound of the FP32-state split path (measured about 2.7e-6)
    assert err <= STATED_F32


@pytest.mark.parametrize("fuse", [2, 3])
def test_box9_full_size_fused_sampled(fuse):
    # The benchmark's launch configuration: the same workload with S sweeps
    # fused per launch plus the edge-band launch; sampled points include the
    # corners and edges, whose values come from the edge-band launch.
    from oracle import tables as T
    dims = (10240, 10240)
    steps = 100
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=dims)
    x0 = synthetic.grid_f32(dims, seed=0)
    with native.Plan("box", 1, w, dims, "f32_split_f16", fuse_steps=fuse) as p:
        info = p.info
        assert info["engine_name"] == "smfmac" and info["fuse_steps"] == fuse
        got = run_plan(p, x0, steps)
    pts = sample_points(*dims, 16, seed=2) + [(0, 4321), (777, 0), (10239, 5), (3, 10238), (1, 1), (10238, 10237)]
    ref = cone_sample(x0, w, steps, pts)
    vals = np.array([got[y, x] for (y, x) in pts], dtype=np.float64)
    err = float(np.abs(vals - ref).max() / np.abs(ref).max())
    s1 = float(np.abs(w).sum())
    ss = float(np.abs(T.compose(np.asarray(w, dtype=np.float64), fuse)).sum())
    b = split_step_bound("f16", n_mma_of(info))
    tol = (steps // fuse) * b * ss + (steps % fuse) * b * s1
    print(f"full-size fused S={fuse} sampled err={err:.3e} tol={tol:.3e}")
    assert err <= tol
    # three fused sweeps per launch reach the split path's 1e-6 (measured
    # about 2e-7); two land at about 7e-7, held to 3e-6 and the FP32 bound
    assert err <= (STATED_SPLIT if fuse == 3 else 3e-6)


FUSED_ZERO = [("box", (64, 64)), ("star", (300, 264)), ("box", (37, 41)), ("box", (3, 5)), ("box", (520, 1030))]


@pytest.mark.parametrize("engine", ["smfmac", "mfma", "direct"])
@pytest.mark.parametrize("shape,dims", FUSED_ZERO)
@pytest.mark.parametrize("fuse,steps", [(2, 6), (2, 7), (3, 6), (3, 7)])
def test_fusion_with_zero_halo(engine, shape, dims, fuse, steps):
    """Fused sweeps on a zero-halo grid (the composed stencil everywhere,
    then the band within r(S-1) of an edge recomputed exactly) against the
    unfused oracle; leftover steps run unfused."""
    from oracle import tables as T
    w, _ = synthetic.random_coeffs(shape, 1, 2, seed=1, grid_shape=dims)
    x0 = synthetic.grid_f32(dims, seed=5)
    with native.Plan(shape, 1, w, dims, "f32_split_f16", boundary="zero", fuse_steps=fuse, engine=engine) as p:
        info = p.info
        assert info["engine_name"] == engine and info["fuse_steps"] == fuse and info["k"] == 2 * fuse + 1
        # the matrix kernels recompute the band inside the sweep launch, the
        # direct engine by a second launch
        assert info["launches_per_sweep"] == (2 if engine == "direct" else 1)
        got = run_plan(p, x0, steps)
    ref = oracle_direct.run(x0.astype(np.float64), w, steps, periodic=False)
    err = normwise_err(got, ref)
    ws = T.compose(np.asarray(w, dtype=np.float64), fuse)
    s1, ss = float(np.abs(w).sum()), float(np.abs(ws).sum())
    fused, rest = steps // fuse, steps % fuse
    if engine == "direct":
        tol = 2 * 2.0 ** -24 * (fused * (np.count_nonzero(ws) + 1) * ss + rest * (np.count_nonzero(w) + 1) * s1)
    else:
        b = split_step_bound("f16", n_mma_of(info))
        tol = fused * b * ss + rest * b * s1
    print(f"engine={engine} {shape} dims={dims} S={fuse} steps={steps} err={err:.3e} tol={tol:.3e}")
    assert err <= tol


MULTI_ITEM = [  # (dims, boundary, fuse, steps): >= 4 work items per workgroup on 256 CUs
    ((2080, 4100), "zero", 1, 6),      # 17 x 65 items, a ragged last band and row block
    ((2080, 4100), "zero", 3, 7),      # two fused launches (plus edge bands), one unfused
    ((2048, 4098), "periodic", 1, 5),  # rows not a multiple of 4 values: 4-byte transfers
    ((2050, 4096), "periodic", 3, 6),  # periodic composed stencil, ragged rows
]


@pytest.mark.parametrize("engine", ["smfmac", "mfma"])
@pytest.mark.parametrize("dims,boundary,fuse,steps", MULTI_ITEM)
def test_multi_item_full_grid(engine, dims, boundary, fuse, steps):
    """The persistent FP32 kernel in its steady state: at least four work
    items per workgroup, so the slab rotation, the items fetched ahead and
    the XCD-interleaved ranges all run, checked point by point against the
    oracle on the whole grid."""
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=dims)
    x0 = synthetic.grid_f32(dims, seed=11)
    with native.Plan("box", 1, w, dims, "f32_split_f16", boundary=boundary, fuse_steps=fuse, engine=engine) as p:
        info = p.info
        assert info["engine_name"] == engine and info["fuse_steps"] == fuse
        got = run_plan(p, x0, steps)
    items = -(-dims[1] // 256) * -(-dims[0] // 32)
    assert items >= 4 * 256
    ref = oracle_direct.run(x0.astype(np.float64), w, steps, periodic=(boundary == "periodic"))
    err = normwise_err(got, ref)
    tol = apriori_bound(info, w, steps, "f32_split_f16")
    print(f"{engine} {dims} {boundary} S={fuse} items={items} err={err:.3e} tol={tol:.3e}")
    assert err <= tol
    assert err <= STATED_F32


@pytest.mark.parametrize("engine,dtype,fuse", [("smfmac", "f32_split_f16", 1), ("smfmac", "f32_split_f16", 3),
                                               ("mfma", "f32_split_bf16", 1), ("direct", "f32", 1),
                                               ("smfmac", "split_bf16", 1)])
def test_sweep_batch_exceeds_cus(engine, dtype, fuse):
    """One launch over 16 grids whose work items together (16 x 165) exceed
    four per compute unit: every grid's result equals its sweep alone, bit
    for bit, and the oracle's within the bound."""
    from .helpers import planes_value
    dims = (1056, 1100) if dtype != "split_bf16" else (1056, 1104)
    boundary = "zero"
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=dims)
    n = 16
    if dtype == "split_bf16":
        hosts = [synthetic.grid_bf16_planes(dims, seed=40 + i) for i in range(n)]
        ins = [torch.from_numpy(h.view(np.int16)).to(DEV) for h in hosts]
        starts = [planes_value(h) for h in hosts]
    else:
        hosts = [synthetic.grid_f32(dims, seed=40 + i) for i in range(n)]
        ins = [torch.from_numpy(h).to(DEV) for h in hosts]
        starts = [h.astype(np.float64) for h in hosts]
    outs = [torch.empty_like(x) for x in ins]
    with native.Plan("box", 1, w, dims, dtype, boundary=boundary, fuse_steps=fuse, engine=engine) as p:
        info = p.info
        assert info["engine_name"] == engine
        p.sweep_batch(ins, outs, stream())
        alone = torch.empty_like(ins[0])
        torch.cuda.synchronize()
        for i in range(n):
            p.sweep(ins[i], alone, stream())
            torch.cuda.synchronize()
            assert torch.equal(alone, outs[i]), f"grid {i} differs from its sweep alone"
        with pytest.raises(native.SparStencilError):
            p.sweep_batch([ins[0], ins[1]], [outs[0], outs[0]], stream())
        with pytest.raises(native.SparStencilError):
            p.sweep_batch([ins[0]], [ins[0]], stream())
    for i in range(n):
        got = outs[i].cpu().numpy()
        got = planes_value(got.view(np.uint16)) if dtype == "split_bf16" else got.astype(np.float64)
        ref = oracle_direct.run(starts[i], w, fuse, periodic=False)
        err = normwise_err(got, ref)
        tol = apriori_bound(info, w, fuse, dtype)
        assert err <= tol, (i, err, tol)


CUSTOM_POINTS = {  # (offsets, coefficients) of patterns neither box nor star
    2: ([(0, 0), (0, -1), (-1, 0), (-1, -1), (0, -2), (2, 1), (1, 2)],
        [0.45, 0.2, 0.15, 0.1, 0.05, 0.03, 0.02]),
    3: ([(0, 0, 0), (0, 0, -1), (0, -1, 0), (-1, 0, 0), (1, 1, 1), (-1, 1, 0)],
        [0.5, 0.15, 0.15, 0.1, 0.05, 0.05]),
    1: ([(0,), (-1,), (-3,), (2,)], [0.6, 0.25, 0.1, 0.05]),
}


@pytest.mark.parametrize("engine", ["smfmac", "mfma", "direct"])
@pytest.mark.parametrize("ndim,dims", [(2, (200, 300)), (2, (129, 131)), (3, (20, 40, 264)), (1, (5000,))])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_custom_points(engine, ndim, dims, boundary):
    """Stencils given as point lists (sparstencil_plan_points, upwind-like
    asymmetric patterns) against the oracle sweeping the box of the same
    points (points_box, itself pinned against the point sum)."""
    from oracle import tables as T
    offs, c = CUSTOM_POINTS[ndim]
    w = T.points_box(offs, c)
    x0 = synthetic.grid_f32(dims, seed=21)
    steps = 5
    with native.Plan("custom", 0, c, dims, "f32_split_f16", boundary=boundary, engine=engine, offsets=offs) as p:
        info = p.info
        assert info["engine_name"] == engine
        kk = len(p.table(native.Q_KERNEL_PERM)) if engine != "direct" else 0
        got = run_plan(p, x0, steps)
    ref = oracle_direct.run(x0.astype(np.float64), w, steps, periodic=(boundary == "periodic"))
    err = normwise_err(got, ref)
    tol = apriori_bound(info, w, steps, "f32_split_f16", kk)
    print(f"custom {ndim}-D {engine} {dims} {boundary} err={err:.3e} tol={tol:.3e}")
    assert err <= tol
