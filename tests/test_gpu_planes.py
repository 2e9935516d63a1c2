"""GPU parity of the bfloat16 hi/lo-plane state (radius 1, radius 3, and two
fused radius-3 sweeps = radius 6) on the sparse, dense and direct engines,
against the FP64 oracle through the C ABI.

The state value is hi + lo (exact in FP64).  Per launch the error relative
to sum|c_S| * max|x| (c_S the coefficients of the launch, composed for a
fused launch) is bounded by the split-product bound of bfloat16 coefficient
parts plus the re-rounding of the result into two planes (u^2 with u = 2^-8);
the tests allow the number of launches times that.  The direct engine adds
FP32 arithmetic over the P points instead of the split products.
"""
import numpy as np
import pytest

import synthetic
from oracle import direct as oracle_direct

from .helpers import cone_sample, normwise_err, sample_points, split_step_bound

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_2506_22969_amd.native")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
U_BF16 = 2.0 ** -8


def planes_value(bits: np.ndarray) -> np.ndarray:
    """(2, ...) uint16 bfloat16 bit patterns -> hi + lo in FP64."""
    f = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return f[0] + f[1]


def run_planes(plan, bits: np.ndarray, steps: int) -> np.ndarray:
    a = torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).to(DEV)
    b = torch.empty_like(a)
    plan.run(a, b, steps, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return b.cpu().numpy().view(np.uint16)


def composed_abs_sum(w: np.ndarray, fuse: int) -> float:
    s = float(np.abs(w).sum())
    return s ** fuse


def tol_planes(info, w, steps, fuse):
    launches = steps // fuse + steps % fuse
    s = composed_abs_sum(w, fuse)
    if info["engine_name"] == "direct":
        p = (2 * info["radius"] + 1) ** 2   # points of the (composed) box
        per = (p + 1) * 2.0 ** -24 * s * 2 + U_BF16 ** 2
    else:
        chunk = 64 if info["engine_name"] == "smfmac" else 32
        n_mma = 3 * info["k_pad"] // chunk
        per = split_step_bound("bf16", n_mma) * s + U_BF16 ** 2
    return launches * per


def coeffs(shape, radius, dims):
    # seeds whose draws are stable on any lattice (checked by random_coeffs)
    seed = {("box", 1): 1, ("star", 3): 45, ("box", 3): 277}[(shape, radius)]
    return synthetic.random_coeffs(shape, radius, 2, seed=seed, grid_shape=dims)[0]


CASES = [  # (shape, radius, fuse, boundary, dims)
    ("box", 1, 1, "zero", (64, 64)),
    ("box", 1, 1, "periodic", (100, 520)),
    ("box", 1, 1, "zero", (300, 264)),
    ("star", 3, 1, "zero", (96, 264)),
    ("box", 3, 1, "periodic", (100, 520)),
    ("star", 3, 2, "periodic", (96, 264)),
    ("box", 3, 2, "periodic", (100, 520)),
    ("star", 3, 2, "periodic", (16, 40)),
    ("box", 1, 1, "periodic", (40, 272)),   # narrowest planes rows for a single wrap
]


@pytest.mark.parametrize("engine", ["smfmac", "mfma", "direct"])
@pytest.mark.parametrize("shape,radius,fuse,boundary,dims", CASES)
def test_planes_small(engine, shape, radius, fuse, boundary, dims):
    w = coeffs(shape, radius, dims)
    bits = synthetic.grid_bf16_planes(dims, seed=3)
    steps = 5
    with native.Plan(shape, radius, w, dims, "split_bf16", boundary=boundary, fuse_steps=fuse,
                     engine=engine) as p:
        info = p.info
        assert info["engine_name"] == engine
        got = run_planes(p, bits, steps)
    ref = oracle_direct.run(planes_value(bits), w, steps, periodic=(boundary == "periodic"))
    err = normwise_err(planes_value(got), ref)
    tol = tol_planes(info, w, steps, fuse)
    print(f"{engine} {shape}{radius} S={fuse} {boundary} {dims} tile=({info['r1']},{info['r2']}) "
          f"err={err:.3e} tol={tol:.3e}")
    assert err <= tol
    # the stored pair is a rounded split: hi = RNE(hi + lo) in bfloat16
    hi = (got[0].astype(np.uint32) << 16).view(np.float32)
    lo = (got[1].astype(np.uint32) << 16).view(np.float32)
    assert np.all(np.abs(lo) <= np.abs(hi) * 2.0 ** -8 + 1e-38)


@pytest.mark.parametrize("engine", ["smfmac", "mfma"])
def test_planes_multi_item_pipeline(engine):
    # 1024 work items: every workgroup runs several pipeline steps
    dims = (4096, 2048)
    w = coeffs("star", 3, dims)
    bits = synthetic.grid_bf16_planes(dims, seed=4)
    steps = 4
    with native.Plan("star", 3, w, dims, "split_bf16", boundary="periodic", fuse_steps=2, engine=engine) as p:
        info = p.info
        got = run_planes(p, bits, steps)
    ref = oracle_direct.run(planes_value(bits), w, steps, periodic=True)
    err = normwise_err(planes_value(got), ref)
    tol = tol_planes(info, w, steps, 2)
    print(f"{engine} multi-item err={err:.3e} tol={tol:.3e}")
    assert err <= tol


def test_planes_fused_equals_unfused_within_bound():
    # two fused sweeps against two single sweeps of the same stencil
    dims = (128, 264)
    w = coeffs("box", 3, dims)
    bits = synthetic.grid_bf16_planes(dims, seed=5)
    with native.Plan("box", 3, w, dims, "split_bf16", boundary="periodic", fuse_steps=2) as p2, \
            native.Plan("box", 3, w, dims, "split_bf16", boundary="periodic") as p1:
        assert p2.launch_count(4) == 2 and p1.launch_count(4) == 4
        a = planes_value(run_planes(p2, bits, 4))
        b = planes_value(run_planes(p1, bits, 4))
    ref = oracle_direct.run(planes_value(bits), w, 4, periodic=True)
    assert normwise_err(a, ref) <= 2 * (split_step_bound("bf16", 18) * composed_abs_sum(w, 2) + U_BF16 ** 2)
    assert normwise_err(b, ref) <= 4 * (split_step_bound("bf16", 12) * composed_abs_sum(w, 1) + U_BF16 ** 2)


@pytest.mark.parametrize("shape", ["star", "box"])
def test_planes_c3_full_size_sampled(shape):
    # Star-2D13P / Box-2D49P, 8192^2 bfloat16 hi+lo planes, 50 sweeps with
    # 2-step fusion, periodic; sampled outputs through their dependency cones.
    dims = (8192, 8192)
    steps = 50
    w = coeffs(shape, 3, dims)
    bits = synthetic.grid_bf16_planes(dims, seed=0)
    with native.Plan(shape, 3, w, dims, "split_bf16", boundary="periodic", fuse_steps=2) as p:
        info = p.info
        assert info["engine_name"] == "smfmac" and info["k"] == 13
        got = run_planes(p, bits, steps)
    x0 = planes_value(bits)
    pts = sample_points(*dims, 6, seed=2)
    ref = cone_sample(x0, w, steps, pts, periodic=True)
    vals = np.array([planes_value(got[:, y, x]) for (y, x) in pts])
    err = float(np.abs(vals - ref).max() / np.abs(ref).max())
    tol = tol_planes(info, w, steps, 2)
    print(f"C3 {shape} sampled err={err:.3e} tol={tol:.3e}")
    assert err <= tol
    # the planes state re-rounds to 16 significant bits every launch, so no
    # stated 1e-6 applies; an empirical ceiling about 3x the measured
    # 1.6e-5 (Star-13) and 2.9e-5 (Box-49) catches a regression the a-priori
    # bound would let through
    assert err <= 1e-4
