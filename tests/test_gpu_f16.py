"""GPU parity of the plain binary16 path (SS_F16): binary16 coefficients and
state, one sparse (or dense) MMA product per K chunk with FP32 accumulation,
each sweep rounded to binary16 -- the paper's FP16 setting (Section 4.1).

The oracle for it is oracle.direct.run_binary16: the same roundings with the
sums formed in FP64.  After one sweep every GPU value is the binary16
rounding of a sum within (n_mma + 1) 2^-24 sum|c x| of the oracle's, so the
two differ by at most one binary16 spacing (where that sum lies near a
rounding boundary, which is rare).  After T sweeps such flips can propagate:
the tests allow T * 2^-9 normwise (four spacings of the largest value per
sweep).  The error against the FP64 oracle is reported as it is (printed),
the path's precision being that of binary16.
"""
import numpy as np
import pytest

import synthetic
from oracle import direct as oracle_direct

from .helpers import cone_sample, normwise_err, sample_points

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_2506_22969_amd.native")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def stream():
    return torch.cuda.current_stream().cuda_stream


def run16(plan, x16: np.ndarray, steps: int) -> np.ndarray:
    a = torch.from_numpy(np.ascontiguousarray(x16)).to(DEV)
    assert a.dtype == torch.float16
    b = torch.empty_like(a)
    plan.run(a, b, steps, stream())
    torch.cuda.synchronize()
    return b.cpu().numpy().astype(np.float64)


def grid16(dims, seed):
    return synthetic.grid_f32(dims, seed=seed).astype(np.float16)


TILES = {1: [("smfmac", 8, 8), ("smfmac", 8, 4), ("smfmac", 16, 4), ("mfma", 8, 8), ("mfma", 8, 4)],
         2: [("smfmac", 8, 8), ("smfmac", 8, 4), ("mfma", 8, 4)],
         3: [("smfmac", 8, 8), ("smfmac", 8, 4), ("mfma", 8, 4)]}
CASES = [(rad, eng, r1, r2) for rad, ts in TILES.items() for (eng, r1, r2) in ts]


@pytest.mark.parametrize("radius,engine,r1,r2", CASES)
@pytest.mark.parametrize("boundary", ["zero", "periodic"])
def test_one_sweep_within_one_spacing(radius, engine, r1, r2, boundary):
    dims = (300, 520)
    w, _ = synthetic.random_coeffs("box", radius, 2, seed=1, grid_shape=dims)
    x16 = grid16(dims, 3)
    with native.Plan("box", radius, w, dims, "f16", boundary=boundary, engine=engine, r1=r1, r2=r2) as p:
        info = p.info
        assert info["engine_name"] == engine and (info["r1"], info["r2"]) == (r1, r2)
        assert info["passes"] == 1
        got = run16(p, x16, 1)
    ref = oracle_direct.run_binary16(x16, w, 1, periodic=(boundary == "periodic"))
    spacing = np.spacing(np.abs(ref).astype(np.float16)).astype(np.float64)
    diff = np.abs(got - ref)
    flips = int(np.count_nonzero(diff))
    print(f"r={radius} {engine} ({r1},{r2}) {boundary}: {flips} of {ref.size} values one spacing off")
    assert np.all(diff <= spacing)
    assert flips <= ref.size // 100


@pytest.mark.parametrize("radius,shape", [(1, "box"), (1, "star"), (3, "box"), (3, "star")])
@pytest.mark.parametrize("engine", ["smfmac", "mfma"])
def test_sweeps_against_binary16_oracle(radius, shape, engine):
    # several work items per workgroup (2080 x 4096: 1040 items), ragged row
    # blocks, zero halo
    dims = (2080, 4096)
    steps = 5
    w, _ = synthetic.random_coeffs(shape, radius, 2, seed=2, grid_shape=dims)
    x16 = grid16(dims, 5)
    with native.Plan(shape, radius, w, dims, "f16", engine=engine) as p:
        info = p.info
        assert info["engine_name"] == engine
        got = run16(p, x16, steps)
    ref16 = oracle_direct.run_binary16(x16, w, steps)
    ref64 = oracle_direct.run(x16.astype(np.float64), w, steps)
    err16 = normwise_err(got, ref16)
    err64 = normwise_err(got, ref64)
    print(f"f16 r={radius} {shape} {engine} ({info['r1']},{info['r2']}) K={info['k_pad']}: "
          f"vs binary16 oracle {err16:.3e}, vs FP64 oracle {err64:.3e} (reported as is)")
    assert err16 <= steps * 2.0 ** -9


def test_periodic_fused_sweeps():
    # two sweeps composed into one radius-2 stencil on a periodic grid: the
    # binary16 path then rounds once per launch, so the oracle is run_binary16
    # of the composed coefficients, once per fused launch
    from oracle import tables as T
    dims = (256, 264)
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=4, grid_shape=dims)
    x16 = grid16(dims, 6)
    with native.Plan("box", 1, w, dims, "f16", boundary="periodic", fuse_steps=2) as p:
        info = p.info
        assert info["fuse_steps"] == 2 and info["k"] == 5
        got = run16(p, x16, 4)
    ws = T.compose(np.asarray(w, dtype=np.float64), 2)
    ref = oracle_direct.run_binary16(x16, ws, 2, periodic=True)
    assert normwise_err(got, ref) <= 2 * 2.0 ** -9


def test_rows_must_be_whole_pieces():
    # binary16 rows move in 16-byte pieces: widths not a multiple of 8 values
    # are refused at plan time
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=(64, 100))
    with pytest.raises(native.SparStencilError):
        native.Plan("box", 1, w, (64, 100), "f16")


def test_constant_field_exact():
    w = synthetic.heat2d_coeffs()
    dims = (96, 160)
    x16 = np.full(dims, 0.75, dtype=np.float16)
    for engine in ("smfmac", "mfma"):
        with native.Plan("star", 1, w, dims, "f16", engine=engine) as p:
            got = run16(p, x16, 3)
        assert np.all(got[3:-3, 3:-3] == 0.75)


def test_full_size_sampled():
    # the Box-2D9P benchmark shape on a binary16 state: 10240^2, 100 sweeps,
    # zero halo, at sampled points through their dependency cones
    dims = (10240, 10240)
    steps = 100
    w, _ = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=dims)
    x16 = grid16(dims, 0)
    with native.Plan("box", 1, w, dims, "f16") as p:
        info = p.info
        assert info["engine_name"] == "smfmac"
        got = run16(p, x16, steps)
    pts = sample_points(*dims, 12, seed=3)
    ref16 = cone_sample(x16, w, steps, pts, binary16=True)
    ref64 = cone_sample(x16, w, steps, pts)
    vals = np.array([got[y, x] for (y, x) in pts])
    e16 = float(np.abs(vals - ref16).max() / np.abs(ref16).max())
    e64 = float(np.abs(vals - ref64).max() / np.abs(ref64).max())
    print(f"f16 full size sampled: vs binary16 oracle {e16:.3e}, vs FP64 oracle {e64:.3e} (reported as is)")
    assert e16 <= steps * 2.0 ** -9
