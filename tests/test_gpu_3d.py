"""GPU parity of the 3-D engines (FP32 state, binary16 or bfloat16 split
products on the sparse and dense matrix cores; the direct FP32 engine)
against the FP64 oracle through the C ABI: Heat-3D 7-point and Box-3D
27-point stencils, zero and periodic boundaries, ragged sizes, several
z chunks per work item, and the 512^3 workload at sampled points.

Tolerances as in the 2-D parity tests: T times the per-sweep split bound
(times sum|c|) for the matrix-core engines, T (P+1) 2^-24 sum|c| for direct.
"""
import numpy as np
import pytest

import synthetic
from oracle import direct as oracle_direct
from oracle.sampling import cone_sample, sample_points3

from .helpers import STATED_SPLIT, normwise_err, split_step_bound

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_2506_22969_amd.native")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def run_plan(plan, x0: np.ndarray, steps: int) -> np.ndarray:
    a = torch.from_numpy(np.ascontiguousarray(x0)).to(DEV)
    b = torch.empty_like(a)
    plan.run(a, b, steps, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return b.cpu().numpy()


def tol_for(info, w, steps, dtype):
    s = float(np.abs(w).sum())
    if info["engine_name"] == "direct":
        return steps * (np.count_nonzero(w) + 1) * 2.0 ** -24 * s * 2
    chunk = 64 if info["engine_name"] == "smfmac" else 32
    n_mma = 3 * info["k_pad"] // chunk
    fmt = "f16" if dtype == "f32_split_f16" else "bf16"
    return steps * split_step_bound(fmt, n_mma) * s


def coeffs(shape):
    # seeds whose draws are stable (checked by random_coeffs)
    seed = {"star": 29, "box": 70}[shape]
    return synthetic.random_coeffs(shape, 1, 3, seed=seed)[0]


CASES = [  # (shape, dims, boundary)
    ("star", (20, 40, 264), "zero"),
    ("box", (20, 40, 264), "periodic"),
    ("box", (7, 33, 129), "zero"),
    ("star", (9, 17, 31), "periodic"),
    ("box", (3, 5, 7), "zero"),
    ("box", (40, 64, 520), "periodic"),
    ("star", (12, 24, 258), "periodic"),   # narrowest rows for a single wrap, 4-byte row transfers
]


@pytest.mark.parametrize("engine", ["smfmac", "mfma", "direct"])
@pytest.mark.parametrize("shape,dims,boundary", CASES)
def test_3d_small(engine, shape, dims, boundary):
    w = coeffs(shape)
    x0 = synthetic.grid_f32(dims, seed=6)
    steps = 4
    with native.Plan(shape, 1, w, dims, "f32_split_f16", boundary=boundary, engine=engine) as p:
        info = p.info
        assert info["engine_name"] == engine
        got = run_plan(p, x0, steps)
    ref = oracle_direct.run(x0.astype(np.float64), w, steps, periodic=(boundary == "periodic"))
    err = normwise_err(got, ref)
    tol = tol_for(info, w, steps, "f32_split_f16")
    print(f"{engine} {shape} {dims} {boundary} err={err:.3e} tol={tol:.3e}")
    assert err <= tol


@pytest.mark.parametrize("engine", ["smfmac", "mfma"])
def test_3d_bf16_parts_and_z_chunks(engine):
    # 2 x 16 columns: the launch splits z into chunks (several items per
    # column, each restarting the plane ring)
    dims = (64, 256, 512)
    w = coeffs("box")
    x0 = synthetic.grid_f32(dims, seed=8)
    steps = 3
    with native.Plan("box", 1, w, dims, "f32_split_bf16", engine=engine) as p:
        info = p.info
        got = run_plan(p, x0, steps)
    ref = oracle_direct.run(x0.astype(np.float64), w, steps)
    err = normwise_err(got, ref)
    tol = tol_for(info, w, steps, "f32_split_bf16")
    print(f"{engine} bf16 z-chunks err={err:.3e} tol={tol:.3e}")
    assert err <= tol


def test_3d_constant_field_bit_exact():
    # Heat-3D (0.25 centre, 0.125 x 6): binary16 coefficients and state 0.5;
    # every product and sum is exact, so interior points stay 0.5
    w = np.zeros((3, 3, 3))
    w[1, 1, 1] = 0.25
    for o in [(0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)]:
        w[o] = 0.125
    dims = (12, 40, 72)
    x0 = np.full(dims, 0.5, dtype=np.float32)
    for engine in ("smfmac", "mfma"):
        with native.Plan("star", 1, w, dims, "f32_split_f16", engine=engine, boundary="periodic") as p:
            assert np.all(run_plan(p, x0, 3) == 0.5)
        with native.Plan("star", 1, w, dims, "f32_split_f16", engine=engine) as p:
            got = run_plan(p, x0, 2)
        assert np.all(got[2:-2, 2:-2, 2:-2] == 0.5)


@pytest.mark.parametrize("shape", ["star", "box"])
def test_3d_c4_full_size_sampled(shape):
    # Heat-3D 7-point / Box-3D 27-point on 512^3 FP32, 20 sweeps, zero halo,
    # binary16 split on the sparse engine; sampled through dependency cones.
    dims = (512, 512, 512)
    steps = 20
    w = coeffs(shape)
    x0 = synthetic.grid_f32(dims, seed=0)
    with native.Plan(shape, 1, w, dims, "f32_split_f16") as p:
        info = p.info
        assert info["engine_name"] == "smfmac"
        got = run_plan(p, x0, steps)
    pts = sample_points3(*dims, 10, seed=3)
    ref = cone_sample(x0, w, steps, pts)
    vals = np.array([got[pt] for pt in pts], dtype=np.float64)
    err = float(np.abs(vals - ref).max() / np.abs(ref).max())
    tol = tol_for(info, w, steps, "f32_split_f16")
    print(f"C4 {shape} sampled err={err:.3e} tol={tol:.3e}")
    assert err <= tol
    # the split path's stated 1e-6 (measured 2e-7 Heat-3D, 6e-7 Box-3D27P)
    assert err <= STATED_SPLIT


FUSED_CASES = [  # (shape, dims, steps): ragged, 4-byte rows, tiny (all band), z chunks
    ("star", (20, 40, 264), 4),
    ("box", (20, 40, 264), 5),
    ("box", (7, 33, 129), 4),
    ("star", (3, 5, 7), 2),
    ("box", (64, 256, 512), 4),
]


@pytest.mark.parametrize("engine", ["smfmac", "mfma", "direct"])
@pytest.mark.parametrize("shape,dims,steps", FUSED_CASES)
def test_3d_fused_zero_halo(engine, shape, dims, steps):
    """Two radius-1 sweeps composed into one radius-2 launch on a zero halo:
    the products (or the direct radius-2 sweep) away from the faces and the
    exact two-sweep band within one of a face, in the same launch; against
    the unfused FP64 oracle.  Odd step counts end with an unfused sweep."""
    from .helpers import apriori_bound
    w = coeffs(shape)
    x0 = synthetic.grid_f32(dims, seed=11)
    with native.Plan(shape, 1, w, dims, "f32_split_f16", fuse_steps=2, engine=engine) as p:
        info = p.info
        assert info["engine_name"] == engine and info["k"] == 5 and info["launches_per_sweep"] == 1
        kk = len(p.table(native.Q_KERNEL_PERM))
        got = run_plan(p, x0, steps)
    ref = oracle_direct.run(x0.astype(np.float64), w, steps)
    err = normwise_err(got, ref)
    tol = apriori_bound(info, w, steps, "f32_split_f16", kk)
    print(f"{engine} {shape} {dims} S=2 T={steps} err={err:.3e} tol={tol:.3e}")
    assert err <= tol


@pytest.mark.parametrize("engine", ["smfmac", "mfma"])
@pytest.mark.parametrize("shape", ["star", "box"])
def test_3d_fused_periodic_bf16(engine, shape):
    """Fused radius-2 launches on a periodic grid (no band) with bfloat16
    parts."""
    from .helpers import apriori_bound
    w = coeffs(shape)
    dims = (24, 48, 264)
    x0 = synthetic.grid_f32(dims, seed=12)
    with native.Plan(shape, 1, w, dims, "f32_split_bf16", fuse_steps=2, boundary="periodic", engine=engine) as p:
        info = p.info
        kk = len(p.table(native.Q_KERNEL_PERM))
        got = run_plan(p, x0, 4)
    ref = oracle_direct.run(x0.astype(np.float64), w, 4, periodic=True)
    err = normwise_err(got, ref)
    tol = apriori_bound(info, w, 4, "f32_split_bf16", kk)
    print(f"{engine} {shape} periodic bf16 S=2 err={err:.3e} tol={tol:.3e}")
    assert err <= tol


@pytest.mark.parametrize("shape", ["star", "box"])
def test_3d_c4_fused_full_size_sampled(shape):
    """C4 shapes (512^3, 20 sweeps, zero halo) with two sweeps per launch on
    the sparse engine, sampled through dependency cones; corners and faces
    are among the points (band values)."""
    from .helpers import apriori_bound
    dims = (512, 512, 512)
    steps = 20
    w = coeffs(shape)
    x0 = synthetic.grid_f32(dims, seed=0)
    with native.Plan(shape, 1, w, dims, "f32_split_f16", fuse_steps=2) as p:
        info = p.info
        assert info["engine_name"] == "smfmac" and info["fuse_steps"] == 2
        kk = len(p.table(native.Q_KERNEL_PERM))
        got = run_plan(p, x0, steps)
    pts = sample_points3(*dims, 12, seed=4) + [(0, 200, 300), (511, 3, 0), (100, 0, 511), (255, 511, 256)]
    ref = cone_sample(x0, w, steps, pts)
    vals = np.array([got[pt] for pt in pts], dtype=np.float64)
    err = float(np.abs(vals - ref).max() / np.abs(ref).max())
    tol = apriori_bound(info, w, steps, "f32_split_f16", kk)
    print(f"C4 fused {shape} sampled err={err:.3e} tol={tol:.3e}")
    assert err <= tol
    assert err <= STATED_SPLIT
