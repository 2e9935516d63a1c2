"""GPU parity of the bfloat16 hi/mid/lo planes state (SS_SPLIT3_BF16): three
bfloat16 planes hold 24 significant bits, the coefficients split three ways,
six products per K chunk (hi*hi, hi*mid, mid*hi, hi*lo, lo*hi, mid*mid)
accumulated in FP32, the result re-split into three planes.

Per launch the error relative to sum|c| * max|x| is bounded by the dropped
products (mid*lo, lo*mid, lo*lo: 3 * 2^-24 with parts at most 2^-8 of the
one before), the coefficients' own split (2^-26), one FP32 rounding per
accumulating product and the FP32 re-split of the result (2^-24): the tests
allow that per launch, with the composed coefficients' sum|c| for fused
launches, and hold every result to the split path's stated 1e-6."""
import numpy as np
import pytest

import synthetic
from oracle import direct as oracle_direct
from oracle import tables as T

from .helpers import STATED_SPLIT, cone_sample, normwise_err

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_2506_22969_amd.native")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def planes3_value(bits: np.ndarray) -> np.ndarray:
    f = (np.asarray(bits).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return f[0] + f[1] + f[2]


def run3(plan, bits, steps):
    a = torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).to(DEV)
    b = torch.empty_like(a)
    plan.run(a, b, steps, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return b.cpu().numpy().view(np.uint16)


def bound(info, w, steps):
    fuse = int(info["fuse_steps"])
    ws = T.compose(np.asarray(w, dtype=np.float64), fuse) if fuse > 1 else np.asarray(w, dtype=np.float64)
    chunk = 64 if info["engine_name"] == "smfmac" else 32
    n_mma = 6 * int(info["k_pad"]) // chunk
    per = (3 * 2.0 ** -24 + 2.0 ** -26 + (n_mma + 1) * 2.0 ** -24)
    s_f, s_1 = float(np.abs(ws).sum()), float(np.abs(w).sum())
    return (steps // fuse) * per * s_f + (steps % fuse) * per * s_1


CASES = [("box", 1, 1, "periodic"), ("box", 1, 1, "zero"), ("star", 3, 1, "zero"), ("box", 3, 2, "periodic"),
         ("star", 3, 2, "periodic")]


@pytest.mark.parametrize("shape,radius,fuse,boundary", CASES)
@pytest.mark.parametrize("engine", ["smfmac", "mfma"])
def test_planes3_against_oracle(shape, radius, fuse, boundary, engine):
    dims = (1056, 4104)            # 33 x 17 row blocks and bands: several items per workgroup, ragged
    steps = 4
    w, _ = synthetic.random_coeffs(shape, radius, 2, seed=45 if radius == 3 else 1, grid_shape=dims)
    bits = synthetic.grid_bf16_planes3(dims, seed=12)
    x0 = planes3_value(bits)
    with native.Plan(shape, radius, w, dims, "split3_bf16", boundary=boundary, fuse_steps=fuse, engine=engine) as p:
        info = p.info
        assert info["engine_name"] == engine and info["passes"] == 6
        got = planes3_value(run3(p, bits, steps))
    ref = oracle_direct.run(x0, w, steps, periodic=(boundary == "periodic"))
    err = normwise_err(got, ref)
    tol = bound(info, w, steps)
    print(f"planes3 {shape} r={radius} S={fuse} {boundary} {engine} ({info['r1']},{info['r2']}) "
          f"K={info['k_pad']} err={err:.3e} tol={tol:.3e}")
    assert err <= tol
    assert err <= STATED_SPLIT


@pytest.mark.parametrize("shape,seed", [("star", 45), ("box", 277)])
def test_planes3_full_size_sampled(shape, seed):
    # the Star-2D13P / Box-2D49P workload on three planes: 8192^2, two fused
    # sweeps per launch, 50 sweeps, periodic; sampled points through their
    # dependency cones, held to the split path's 1e-6
    dims = (8192, 8192)
    steps = 50
    w, _ = synthetic.random_coeffs(shape, 3, 2, seed=seed, grid_shape=dims)
    bits = synthetic.grid_bf16_planes3(dims, seed=0)
    with native.Plan(shape, 3, w, dims, "split3_bf16", boundary="periodic", fuse_steps=2) as p:
        info = p.info
        assert info["engine_name"] == "smfmac"
        out = run3(p, bits, steps)
    pts = [(0, 0), (4095, 17), (8191, 8191), (1234, 6543), (77, 8000), (6000, 3)]
    x0 = planes3_value(bits)
    ref = cone_sample(x0, w, steps, pts, periodic=True)
    vals = np.array([planes3_value(out[:, y, x]) for (y, x) in pts])
    err = float(np.abs(vals - ref).max() / np.abs(ref).max())
    print(f"planes3 full size {shape}: ({info['r1']},{info['r2']}) err={err:.3e} tol={bound(info, w, steps):.3e}")
    assert err <= bound(info, w, steps)
    assert err <= STATED_SPLIT
