"""Benchmark: Box-2D9P on a 10240 x 10240 FP32 grid, 100 sweeps, zero halo,
binary16 hi+lo split products on gfx950 sparse MFMA (SMFMAC).

One step = one sparstencil_run of the whole workload (100 sweeps) on grids
already resident in HBM; by default three sweeps are fused per launch (the
composed stencil, with the band within 2r of the edges recomputed exactly by
the same launch), as the paper fuses three sweeps.  Prints one JSON line
with GStencil/s (paper Section 4.1, Eq. 12: T * prod(N_i) / (t * 1e9)),
latency percentiles, the dense-MFMA and direct-FMA engines on the same
workload (fused and unfused), the roofline of the sparse sweep launch (HIP
events on its stream) and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NY = NX = 10240
SWEEPS = 100
HBM_PEAK_GBS = 8000.0
BYTES_PER_POINT = 8  # FP32 state: one 4-byte read and one 4-byte write per point-sweep
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_smfmac_box2d9p_10240.json")
# sources of the sparse 2-D sweep kernel the traffic figure was measured on
KERNEL_SRCS = [os.path.join(ROOT, "paper_2506_22969_amd", "csrc", f)
               for f in ("mma2d_conv.hpp", "mma2d_impl.hpp", "mma2d_f32_r1.hip", "mma2d_f32_r3.hip", "kgeom.hpp",
                         "kargs.hpp")]
SMFMAC_SPEC_TFLOPS = 5000.0   # dense-equivalent binary16 sparse peak (2x the dense 2.5 PF)
MFMA_SPEC_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--engines", default="smfmac,mfma,direct",
                    help="engines to time; the first is the headline")
    ap.add_argument("--fuse", type=int, default=3, choices=[1, 2, 3],
                    help="sweeps fused per launch on the headline workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--sweep-loop", type=int, default=40, help="sweeps timed for the roofline")
    ap.add_argument("--serve-jobs", type=int, default=2000,
                    help="jobs of the serving-mix leg (0 skips it)")
    ap.add_argument("--serve-loads", default="0.5,0.7,0.9",
                    help="Poisson arrival rates as fractions of the measured batch capacity")
    ap.add_argument("--no-layouts", dest="layouts", action="store_false",
                    help="skip the measured sweep over the instantiated tiles")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other workloads (Heat-2D FP64, radius-3 bfloat16 planes, 3-D)")
    ap.add_argument("--profile", choices=["box2d9p", "box2d49p_planes", "box3d27p", "heat3d7p", "heat1d3p", "1d5p"],
                    help="only copy the grid once and run four sweeps of one workload on the sparse engine (for profilers)")
    return ap.parse_args()


def kernel_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_entry(fuse: int, tile):
    """Measured HBM bytes per launch, only if taken on the current kernel
    source, fusion and tile."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_sha256_16") != kernel_hash() or t.get("fuse_steps", 1) != fuse
            or t.get("tile") != list(tile)):
        return None
    return t.get("bytes_per_launch")


def time_engine(native, torch, w, x0_dev, engine, steps, warmup, stream, fuse):
    plan = native.Plan("box", 1, w, (NY, NX), "f32_split_f16", engine=engine, fuse_steps=fuse)
    info = plan.info
    a = torch.empty_like(x0_dev)
    b = torch.empty_like(x0_dev)
    for _ in range(warmup):
        a.copy_(x0_dev)
        plan.run(a, b, SWEEPS, stream.cuda_stream)
    torch.cuda.synchronize()
    lat = []
    t_total = 0.0
    for _ in range(steps):
        a.copy_(x0_dev)  # each step starts from the same resident input
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        plan.run(a, b, SWEEPS, stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t_total += time.perf_counter() - t0
        lat.append(e0.elapsed_time(e1))
    return plan, info, np.array(lat), t_total, b


def sweep_roofline(torch, plan, x0_dev, stream, n):
    """Average duration of one sweep kernel: HIP events around n back-to-back
    sweeps on the stream they are launched on."""
    a = x0_dev.clone()
    b = torch.empty_like(a)
    for _ in range(4):
        plan.sweep(a, b, stream.cuda_stream)
        a, b = b, a
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(n):
        plan.sweep(a, b, stream.cuda_stream)
        a, b = b, a
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def measured_peaks(native, torch, stream):
    """Peaks measured on this device: HBM bandwidth of a plain 4 GiB
    device-to-device copy (read + write bytes), and the matrix-core probe's
    dense-equivalent binary16 rate, sparse and dense (HIP events)."""
    n = 1 << 30
    a = torch.empty(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 5
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    hbm = 2 * 4 * n * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    out = {"hbm_copy_gbs": round(hbm, 1)}
    wgs = 256 * 8
    buf = torch.empty(wgs * 256 * 4, dtype=torch.float32, device="cuda:0")
    for eng in ("smfmac", "mfma"):
        native.sparstencil_probe_mma_peak(eng, 50, wgs, buf, stream.cuda_stream)
        torch.cuda.synchronize()
        e0.record(stream)
        flops = native.sparstencil_probe_mma_peak(eng, 2000, wgs, buf, stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        out[f"{eng}_tflops"] = round(flops / (e0.elapsed_time(e1) / 1e3) / 1e12, 1)
    return out


def issued_mma(info) -> int:
    """Matrix products one 2-D sweep launch issues: every work item (256 x 32
    outputs) runs 8 waves x 4 M-block units (U * MB = 4 for every tile) x K
    chunks x passes."""
    items = -(-NX // 256) * -(-NY // 32)
    chunk = 64 if info["engine_name"] == "smfmac" else 32
    return items * 32 * (info["k_pad"] // chunk) * info["passes"]


def layout_sweep(native, torch, w, x0_dev, stream, n):
    """Layout exploration measured (paper Section 3.3, Eqs. 6-11; Section
    4.5): every instantiated sparse tile of the headline launch (three fused
    sweeps, k = 7) and of the unfused sweep (k = 3), its modelled time T and
    its measured sweep time; the model's pick is the plan's default."""
    rows = []
    for fuse, tiles in ((3, [(8, 8), (8, 4), (16, 2), (8, 2)]), (1, [(8, 8), (16, 4), (8, 4), (16, 2), (8, 2)])):
        with native.Plan("box", 1, w, (NY, NX), "f32_split_f16", engine="smfmac", fuse_steps=fuse) as p0:
            pick = (p0.info["r1"], p0.info["r2"])
            model = {(int(r[0]), int(r[1])): r for r in p0.table(native.Q_MODEL).reshape(-1, 7)}
        for t in tiles:
            with native.Plan("box", 1, w, (NY, NX), "f32_split_f16", engine="smfmac", fuse_steps=fuse,
                             r1=t[0], r2=t[1]) as p:
                ms = sweep_roofline(torch, p, x0_dev, stream, n)
                kp = int(p.table(native.Q_KERNEL_PERM).size)   # the kernel's own K
            m = model.get(t)
            rows.append({"workload": "box radius 1 FP32 10240^2", "fuse_steps": fuse, "tile": list(t), "k_pad": kp,
                         "model_t_us": None if m is None else
                         round(m[2] * 1e6, 2), "measured_us": round(ms * 1e3, 2), "model_pick": t == pick})
    # the radius-3 stencils on bfloat16 planes, two fused sweeps (k = 13)
    import synthetic
    bits = synthetic.grid_bf16_planes((8192, 8192), seed=0)
    xp = torch.from_numpy(bits.view(np.int16)).to("cuda:0")
    del bits
    for shape, seed in (("star", 45), ("box", 277)):
        wp = synthetic.random_coeffs(shape, 3, 2, seed=seed, grid_shape=(8192, 8192))[0]
        with native.Plan(shape, 3, wp, (8192, 8192), "split_bf16", boundary="periodic", fuse_steps=2,
                         engine="smfmac") as p0:
            pick = (p0.info["r1"], p0.info["r2"])
            model = {(int(r[0]), int(r[1])): r for r in p0.table(native.Q_MODEL).reshape(-1, 7)}
        for t in ((16, 2), (16, 1), (8, 4), (8, 2)):
            with native.Plan(shape, 3, wp, (8192, 8192), "split_bf16", boundary="periodic", fuse_steps=2,
                             engine="smfmac", r1=t[0], r2=t[1]) as p:
                ms = sweep_roofline(torch, p, xp, stream, n)
                kp = int(p.table(native.Q_KERNEL_PERM).size)   # the kernel's own K
            m = model.get(t)
            rows.append({"workload": f"{shape} radius 3 bf16 planes 8192^2", "fuse_steps": 2, "tile": list(t),
                         "k_pad": kp, "model_t_us": None if m is None else round(m[2] * 1e6, 2),
                         "measured_us": round(ms * 1e3, 2), "model_pick": t == pick})
    del xp
    torch.cuda.empty_cache()
    return rows


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x0: np.ndarray, w: np.ndarray, gpu_out: np.ndarray, budget_s: float):
    """The FP64 oracle on the host cores: full-grid sweeps for about budget_s
    seconds on all the threads OpenMP gives it (throughput), a third as long
    on one thread, then sampled outputs of the 100-sweep run through their
    dependency cones (error of the GPU result)."""
    from oracle import direct as oracle_direct
    from oracle.sampling import cone_sample, sample_points

    xd = x0.astype(np.float64)

    def rate(seconds, nthreads):
        # runs of one sweep (the first also warms the thread pool) until
        # `seconds` of sweeping have been timed
        oracle_direct.run(xd, w, 1, nthreads=nthreads)
        n, dt = 0, 0.0
        while dt < seconds:
            t0 = time.perf_counter()
            oracle_direct.run(xd, w, 1, nthreads=nthreads)
            dt += time.perf_counter() - t0
            n += 1
        return n, dt, n * NY * NX / dt / 1e9

    n, dt, value = rate(budget_s, 0)
    n1, dt1, value1 = rate(budget_s / 3, 1)
    pts = sample_points(NY, NX, 16, seed=1)
    ref = cone_sample(x0, w, SWEEPS, pts)
    vals = np.array([gpu_out[y, x] for (y, x) in pts], dtype=np.float64)
    err = float(np.abs(vals - ref).max() / np.abs(ref).max())
    return {"value": value, "unit": "GStencil/s", "cores": oracle_direct.threads(),
            "kind": "oracle",
            "sample": f"{n} full-grid FP64 sweeps of the 10240^2 Box-2D9P grid ({dt:.1f} s); "
                      f"error check on 16 sampled outputs of the 100-sweep run via dependency cones",
            "single_thread": {"value": value1, "unit": "GStencil/s", "cores": 1,
                              "sample": f"{n1} full-grid FP64 sweeps on one thread ({dt1:.1f} s)"},
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}, err


def timed_run(torch, plan, x_dev, steps, stream, reps=1):
    """Milliseconds of plan.run over `steps` sweeps (HIP events, median of
    reps after one warm-up) and the output of the last run."""
    a = torch.empty_like(x_dev)
    b = torch.empty_like(x_dev)
    a.copy_(x_dev)
    plan.run(a, b, steps, stream.cuda_stream)
    ms = []
    for _ in range(reps):
        a.copy_(x_dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.run(a, b, steps, stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms)), b


def workloads_leg(native, torch, stream):
    """The other workloads of the study on every engine that runs them:
    Heat-2D 256^2 FP64 (10 sweeps, zero halo), Star-2D13P / Box-2D49P on
    8192^2 bfloat16 hi+lo planes (50 sweeps, 2-step fusion, periodic),
    Heat-3D / Box-3D27P on 512^3 FP32 (20 sweeps, zero halo, one or two
    sweeps per launch) and 3- and
    5-point 1-D stencils on 10,240,000 points (100 sweeps, zero halo, one or
    three sweeps per launch).  Returns the
    timings and, per result, the inputs and GPU values at sampled points for
    the oracle check."""
    import synthetic

    out, checks = {}, []

    def record(name, shape, radius, w, dims, dtype, steps, engines, x_host, make_dev, periodic,
               fuse=1, reps=3, pts=None, pick=None):
        x_dev = make_dev(x_host)
        entry = {}
        for eng in engines:
            with native.Plan(shape, radius, w, dims, dtype, boundary="periodic" if periodic else "zero",
                             fuse_steps=fuse, engine=eng) as p:
                info = p.info
                ms, y = timed_run(torch, p, x_dev, steps, stream, reps)
                pts_vals = None
                if pts is not None:
                    pts_vals = [pick(y, pt) for pt in pts]
            points = int(np.prod(dims))
            entry[eng] = {"gstencil_s": round(steps * points / ms / 1e6, 2), "ms_per_run": round(ms, 3),
                          "tile": [info["r1"], info["r2"]], "k_pad": info["k_pad"]}
            if pts is not None:
                checks.append((name, eng, shape, radius, w, x_host, steps, periodic, pts, pts_vals, dtype))
        out[name] = entry
        del x_dev
        torch.cuda.empty_cache()

    # Heat-2D 256^2 FP64: the whole grid is small enough for a full oracle run
    w = synthetic.heat2d_coeffs()
    x = synthetic.grid_f64((256, 256), seed=0)
    record("heat2d_256_f64_T10", "star", 1, w, (256, 256), "f64", 10, ["direct", "mfma"], x,
           lambda h: torch.from_numpy(h).to("cuda:0"), False, reps=21, pts=[None],
           pick=lambda y, pt: y.cpu().numpy())
    # radius-3 stencils on bfloat16 planes, two fused sweeps per launch
    bits = synthetic.grid_bf16_planes((8192, 8192), seed=0)
    for name, shape, seed in [("star2d13p_8192_planes_S2_T50", "star", 45), ("box2d49p_8192_planes_S2_T50", "box", 277)]:
        w = synthetic.random_coeffs(shape, 3, 2, seed=seed, grid_shape=(8192, 8192))[0]
        pts = [(0, 0), (4095, 17), (8191, 8191), (1234, 6543)]
        record(name, shape, 3, w, (8192, 8192), "split_bf16", 50, ["smfmac", "mfma", "direct"], bits,
               lambda h: torch.from_numpy(h.view(np.int16)).to("cuda:0"), True, fuse=2, pts=pts,
               pick=lambda y, pt: y[:, pt[0], pt[1]].cpu().numpy().view(np.uint16).copy())
    del bits
    # the same two stencils on bfloat16 hi, mid and lo planes (24 significant
    # bits, six products per K chunk)
    bits3 = synthetic.grid_bf16_planes3((8192, 8192), seed=0)
    for name, shape, seed in [("star2d13p_8192_planes3_S2_T50", "star", 45), ("box2d49p_8192_planes3_S2_T50", "box", 277)]:
        w = synthetic.random_coeffs(shape, 3, 2, seed=seed, grid_shape=(8192, 8192))[0]
        pts = [(0, 0), (4095, 17), (8191, 8191), (1234, 6543)]
        record(name, shape, 3, w, (8192, 8192), "split3_bf16", 50, ["smfmac", "mfma"], bits3,
               lambda h: torch.from_numpy(h.view(np.int16)).to("cuda:0"), True, fuse=2, pts=pts,
               pick=lambda y, pt: y[:, pt[0], pt[1]].cpu().numpy().view(np.uint16).copy())
    del bits3
    # the headline Box-2D9P shape on a plain binary16 state (the paper's FP16
    # setting): 10240^2, 100 sweeps, zero halo, one sweep per launch
    w = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=(NY, NX))[0]
    x16 = synthetic.grid_f32((NY, NX), seed=0).astype(np.float16)
    record("box2d9p_10240_f16_T100", "box", 1, w, (NY, NX), "f16", SWEEPS, ["smfmac", "mfma"], x16,
           lambda h: torch.from_numpy(h).to("cuda:0"), False, pts=sample_points_2d(NY, NX, 8),
           pick=lambda y, pt: float(y[pt].item()))
    del x16
    # 3-D 512^3 FP32, one sweep per launch and two fused sweeps per launch
    # (the band within one of a face recomputed in the same launch)
    x3 = synthetic.grid_f32((512, 512, 512), seed=0)
    for name, shape, seed, fuse in [("heat3d7p_512_T20", "star", 29, 1), ("box3d27p_512_T20", "box", 70, 1),
                                    ("heat3d7p_512_S2_T20", "star", 29, 2), ("box3d27p_512_S2_T20", "box", 70, 2)]:
        w = synthetic.random_coeffs(shape, 1, 3, seed=seed)[0]
        pts = [(0, 0, 0), (255, 100, 511), (511, 511, 3), (17, 300, 200), (0, 250, 250)]
        record(name, shape, 1, w, (512, 512, 512), "f32_split_f16", 20, ["smfmac", "mfma", "direct"], x3,
               lambda h: torch.from_numpy(h).to("cuda:0"), False, fuse=fuse, pts=pts,
               pick=lambda y, pt: float(y[pt].item()))
    del x3
    # 1-D on the paper's 10,240,000-point grids: a 3-point (Heat-1D shape)
    # and a 5-point stencil, 100 sweeps with a zero halo, one sweep per
    # launch and three fused sweeps per launch (plus the end-band launch)
    n1 = 10_240_000
    x1 = synthetic.grid_f32((n1,), seed=0)
    for name, radius, fuse in [("heat1d3p_10240000_T100", 1, 1), ("heat1d3p_10240000_S3_T100", 1, 3),
                               ("1d5p_10240000_T100", 2, 1), ("1d5p_10240000_S3_T100", 2, 3)]:
        w = synthetic.random_coeffs("box", radius, 1, seed=3, grid_shape=(4096,))[0]
        pts = [(0,), (4096,), (5_000_000,), (n1 - 1,)]
        record(name, "box", radius, w, (n1,), "f32_split_f16", 100, ["smfmac", "mfma", "direct"], x1,
               lambda h: torch.from_numpy(h).to("cuda:0"), False, fuse=fuse, reps=5, pts=pts,
               pick=lambda y, pt: float(y[pt].item()))
    return out, checks


def sample_points_2d(ny, nx, n):
    from oracle.sampling import sample_points
    return sample_points(ny, nx, n, seed=5)


def check_workloads(checks):
    """Oracle side of workloads_leg: normwise error of each engine's result
    at its sampled points (the whole grid for Heat-2D)."""
    from oracle import direct as oracle_direct
    from oracle.sampling import cone_sample

    errs = {}
    cache = {}
    for name, eng, shape, radius, w, x_host, steps, periodic, pts, vals, dtype in checks:
        if dtype == "f64":
            key = (name,)
            if key not in cache:
                cache[key] = oracle_direct.run(x_host, w, steps, periodic=periodic)
            ref = cache[key]
            got = vals[0]
            err = float(np.abs(got - ref).max() / np.abs(ref).max())
        else:
            key = (name, "cones")
            if key not in cache:
                if dtype in ("split_bf16", "split3_bf16"):
                    f = (x_host.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
                    x0 = f.sum(axis=0)
                else:
                    x0 = x_host
                cache[key] = cone_sample(x0, w, steps, pts, periodic=periodic)
            ref = cache[key]
            if dtype in ("split_bf16", "split3_bf16"):
                got = np.array([float((v.astype(np.uint32) << 16).view(np.float32).astype(np.float64).sum())
                                for v in vals])
            else:
                got = np.array(vals, dtype=np.float64)
            err = float(np.abs(got - ref).max() / np.abs(ref).max())
            if dtype == "f16":
                # reported as it is against FP64, and against the binary16
                # computation the path defines
                key16 = (name, "cones16")
                if key16 not in cache:
                    cache[key16] = cone_sample(x_host, w, steps, pts, periodic=periodic, binary16=True)
                r16 = cache[key16]
                err = {"error_vs_oracle": err,
                       "error_vs_binary16_oracle": float(np.abs(got - r16).max() / np.abs(r16).max())}
        errs.setdefault(name, {})[eng] = err
    return errs


SERVE_DTYPES = {"f32": "f32_split_f16", "split_bf16": "f32_split_bf16"}


def serving_leg(native, torch, n_jobs: int, loads):
    """Serving mix: jobs of several stencils, sizes, step counts and dtypes
    through one server (2-D radius-1 and 1-D jobs with three sweeps fused
    per launch).  Passes over the same jobs: all submitted at once (batch
    capacity), one job at a time through sparstencil_run, and Poisson
    arrivals at each of `loads` x the batch capacity (latency percentiles
    from arrival to result).  The server's arena is the free HBM
    (hipMemGetInfo, through torch) less a margin."""
    import synthetic

    jobs = synthetic.job_stream(n_jobs, rate_per_s=1.0)
    dev = "cuda:0"
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    plans, inputs, sinks, coeffs = {}, {}, {}, {}
    for j in jobs:
        key = (j["kind"], j["grid"], j["dtype"], j["coeff_seed"])
        if key not in plans:
            # every grid of the mix exceeds the stability check's per-axis
            # lattice cap, so one draw per (stencil, seed) serves all sizes
            ck = (j["kind"], j["coeff_seed"])
            if ck not in coeffs:
                coeffs[ck] = synthetic.random_coeffs(j["shape"], j["radius"], j["ndim"], seed=j["coeff_seed"],
                                                     grid_shape=j["grid"])[0]
            # 2-D radius-1 and 1-D jobs fuse three sweeps per launch (zero
            # halo, edge band recomputed), as the headline workload does
            fuse = 3 if (j["ndim"] == 2 and j["radius"] == 1) or (j["ndim"] == 1 and 3 * j["radius"] <= 8) else 1
            plans[key] = native.Plan(j["shape"], j["radius"], coeffs[ck], j["grid"], SERVE_DTYPES[j["dtype"]],
                                     fuse_steps=fuse)
        if j["grid"] not in inputs:
            inputs[j["grid"]] = torch.rand(j["grid"], generator=gen, device=dev, dtype=torch.float32)
            sinks[j["grid"]] = torch.empty_like(inputs[j["grid"]])
        j["plan"] = plans[key]
        j["points"] = int(np.prod(j["grid"]))
    total_ps = sum(j["points"] * j["steps"] for j in jobs)
    torch.cuda.synchronize()
    free, total_hbm = torch.cuda.mem_get_info()
    # admission by the HBM left after the inputs: the free bytes less a
    # margin of 5% of the device (at least 8 GiB) for the runtime and torch
    margin = max(8 << 30, total_hbm // 20)
    arena_bytes = (free - margin) // (1 << 20) * (1 << 20)
    largest = max(p.grid_bytes for p in plans.values())
    if arena_bytes < 4 * largest:
        raise RuntimeError(f"free HBM ({free} B) leaves no room for the serving arena")
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def batch(srv):
        t0 = srv.clock()
        ids = [srv.submit(j["plan"], inputs[j["grid"]], sinks[j["grid"]], j["steps"]) for j in jobs]
        srv.drain()
        return srv.clock() - t0, ids

    with native.Server(arena, arena_bytes, max_jobs=n_jobs, num_streams=4) as srv:
        _, ids = batch(srv)  # warm-up: first launches of every kernel variant
        for jid in ids:
            srv.release(jid)
        makespan, ids = batch(srv)
        for jid in ids:
            srv.release(jid)
        capacity = n_jobs / makespan
        open_loop = []
        for load in loads:
            arrivals = synthetic.job_stream(n_jobs, rate_per_s=load * capacity)
            ids = []
            t0 = time.perf_counter()
            for j, a in zip(jobs, arrivals):
                wait = a["arrival"] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                ids.append(srv.submit(j["plan"], inputs[j["grid"]], sinks[j["grid"]], j["steps"]))
            srv.drain()
            lat = []
            for jid in ids:
                st, info = srv.poll(jid)
                if st != native.SS_OK:
                    raise RuntimeError(f"serving job failed: {native.status_string(st)}")
                lat.append((info["t_done"] - info["t_submit"]) * 1e3)
                srv.release(jid)
            span = time.perf_counter() - t0
            lat = np.array(lat)
            open_loop.append({"load": load, "gstencil_s": round(total_ps / span / 1e9, 2),
                              "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                                             "p99": round(float(np.percentile(lat, 99)), 3)}})
            print(f"serving load {load}: p50 {open_loop[-1]['latency_ms']['p50']} ms, "
                  f"p99 {open_loop[-1]['latency_ms']['p99']} ms", file=sys.stderr, flush=True)

    # one job at a time through sparstencil_run on one stream
    stream = torch.cuda.current_stream()
    scratch = {g: torch.empty_like(x) for g, x in inputs.items()}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in jobs:
        a = scratch[j["grid"]]
        a.copy_(inputs[j["grid"]])
        j["plan"].run(a, sinks[j["grid"]], j["steps"], stream.cuda_stream)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    for p in plans.values():
        p.close()
    mid = min(open_loop, key=lambda r: abs(r["load"] - 0.7))
    return {
        "jobs": n_jobs,
        "mix": "Poisson stream over 1D 5-point 2^20, 2D 5/9/13-point 1024^2-8192^2, 3D 7/27-point "
               "128^3-384^3, steps U{10..200}, FP32 state with binary16 or bfloat16 split products, "
               "4 coefficient seeds per stencil",
        "point_steps": total_ps,
        "batch_gstencil_s": round(total_ps / makespan / 1e9, 2),
        "one_at_a_time_gstencil_s": round(total_ps / seq / 1e9, 2),
        "capacity_jobs_s": round(capacity, 2),
        "open_loop": open_loop,
        "load": mid["load"],
        "latency_ms": mid["latency_ms"],
        "arena_gib": round(arena_bytes / 2 ** 30, 2),
        "arena_rule": "free HBM at server start (hipMemGetInfo) less max(8 GiB, 5% of the device)",
    }


def profile_only(name: str, fuse: int):
    """One grid copy and four sweeps of one workload on the sparse engine,
    nothing else: a short program for counter collection."""
    import torch

    import synthetic
    from paper_2506_22969_amd import native

    stream = torch.cuda.current_stream()
    if name == "box2d9p":
        w = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=(NY, NX))[0]
        x = torch.from_numpy(synthetic.grid_f32((NY, NX), seed=0)).to("cuda:0")
        plan = native.Plan("box", 1, w, (NY, NX), "f32_split_f16", engine="smfmac", fuse_steps=fuse)
    elif name == "box2d49p_planes":
        w = synthetic.random_coeffs("box", 3, 2, seed=277, grid_shape=(8192, 8192))[0]
        bits = synthetic.grid_bf16_planes((8192, 8192), seed=0)
        x = torch.from_numpy(bits.view(np.int16)).to("cuda:0")
        plan = native.Plan("box", 3, w, (8192, 8192), "split_bf16", boundary="periodic", fuse_steps=2,
                           engine="smfmac")
    elif name in ("heat1d3p", "1d5p"):
        radius = 1 if name == "heat1d3p" else 2
        w = synthetic.random_coeffs("box", radius, 1, seed=3, grid_shape=(4096,))[0]
        x = torch.from_numpy(synthetic.grid_f32((10_240_000,), seed=0)).to("cuda:0")
        plan = native.Plan("box", radius, w, (10_240_000,), "f32_split_f16", engine="smfmac")
    else:
        shape, seed = ("box", 70) if name == "box3d27p" else ("star", 29)
        w = synthetic.random_coeffs(shape, 1, 3, seed=seed)[0]
        x = torch.from_numpy(synthetic.grid_f32((512, 512, 512), seed=0)).to("cuda:0")
        plan = native.Plan(shape, 1, w, (512, 512, 512), "f32_split_f16", engine="smfmac", fuse_steps=min(fuse, 2))
    y = torch.empty_like(x)
    # one device copy of the grid: a plain copy kernel of known size, which
    # calibrates the HBM byte counters
    y.copy_(x)
    torch.cuda.synchronize()
    for _ in range(4):
        plan.sweep(x, y, stream.cuda_stream)
        x, y = y, x
    torch.cuda.synchronize()
    info = plan.info
    plan.close()
    print(json.dumps({"profile": name, "tile": [info["r1"], info["r2"]], "k_pad": info["k_pad"]}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the stencil path runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.profile:
        profile_only(args.profile, args.fuse)
        return
    import torch

    import synthetic
    from paper_2506_22969_amd import native

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    w, cseed = synthetic.random_coeffs("box", 1, 2, seed=1, grid_shape=(NY, NX))
    x0 = synthetic.grid_f32((NY, NX), seed=0)
    x0_dev = torch.from_numpy(x0).to("cuda:0")

    engines = [e for e in args.engines.split(",") if e]
    results = {}
    head = None
    unfused = {}
    for i, eng in enumerate(engines):
        steps = args.steps if i == 0 else max(2, args.steps // 3)
        plan, info, lat, t_total, out = time_engine(native, torch, w, x0_dev, eng, steps, args.warmup, stream,
                                                    args.fuse)
        gst = SWEEPS * NY * NX / (t_total / steps) / 1e9
        results[eng] = {"gstencil_s": round(gst, 2), "ms_per_run": round(t_total / steps * 1e3, 3),
                        "tile": [info["r1"], info["r2"]], "k_pad": info["k_pad"],
                        "fuse_steps": info["fuse_steps"], "plan_ms": round(info["plan_seconds"] * 1e3, 3)}
        if i == 0:
            head = (plan, info, lat, t_total, steps, out.cpu().numpy())
        else:
            plan.close()
        if args.fuse > 1:
            # the same engine one sweep per launch, for comparison
            p1, i1, _, t1, _ = time_engine(native, torch, w, x0_dev, eng, max(2, args.steps // 3), 1, stream, 1)
            unfused[eng] = {"gstencil_s": round(SWEEPS * NY * NX / (t1 / max(2, args.steps // 3)) / 1e9, 2),
                            "tile": [i1["r1"], i1["r2"]], "k_pad": i1["k_pad"]}
            if i == 0:
                unfused[eng]["sweep_ms"] = round(sweep_roofline(torch, p1, x0_dev, stream, args.sweep_loop), 4)
            p1.close()
        sys.stdout.flush()
    plan, info, lat, t_total, steps, gpu_out = head
    ms = t_total / steps * 1e3
    value = SWEEPS * NY * NX / (ms / 1e3) / 1e9

    sweep_ms = sweep_roofline(torch, plan, x0_dev, stream, args.sweep_loop)
    alg_bytes = BYTES_PER_POINT * NY * NX
    achieved = alg_bytes / (sweep_ms / 1e3) / 1e9
    peaks = measured_peaks(native, torch, stream)
    mma_flops = issued_mma(info) * 2.0 * 16 * 16 * 64
    mma_tf = mma_flops / (sweep_ms / 1e3) / 1e12
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_entry(args.fuse, (info["r1"], info["r2"])),
            "kernel": f"k_mma2c (sparse, binary16 split, tile {info['r1']}x{info['r2']})" +
                      (f", {args.fuse} sweeps per launch, the edge band computed in the launch" if args.fuse > 1 else ""),
            "sweep_ms": round(sweep_ms, 4), "algorithmic_bytes_per_launch": alg_bytes,
            "frac_of_measured_hbm": round(achieved / peaks["hbm_copy_gbs"], 4),
            "smfmac": {"issued_dense_equiv_flops_per_launch": mma_flops, "achieved_tflops": round(mma_tf, 1),
                       "frac_of_spec": round(mma_tf / SMFMAC_SPEC_TFLOPS, 4),
                       "frac_of_measured": round(mma_tf / peaks["smfmac_tflops"], 4),
                       "useful_tflops": round(2 * info["k"] ** 2 * NY * NX / (sweep_ms / 1e3) / 1e12, 2)},
            "measured_peaks": peaks}
    if unfused.get(engines[0], {}).get("sweep_ms"):
        u_ms = unfused[engines[0]]["sweep_ms"]
        unfused[engines[0]]["roofline_frac"] = round(alg_bytes / (u_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    plan.close()

    line = {
        "metric": "GStencil/s + % HBM/SMFMAC peak vs dense-MFMA/direct at stated error; p99 lat",
        "value": round(value, 2), "unit": "GStencil/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "Box-2D9P 10240x10240 FP32 state, binary16 hi+lo split products "
                               "with FP32 accumulation, 100 sweeps, zero halo",
                   "engine": engines[0], "fuse_steps": info["fuse_steps"],
                   "tile": [info["r1"], info["r2"]], "k_pad": info["k_pad"],
                   "coeff_seed": cseed, "grid_seed": 0, "accumulate": "f32"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3)},
        "engines": results,
        "engines_unfused": unfused,
        "roofline": roof,
    }
    if args.layouts:
        line["layout_sweep"] = layout_sweep(native, torch, w, x0_dev, stream, max(8, args.sweep_loop // 4))
    del x0_dev
    torch.cuda.empty_cache()
    checks = []
    if not args.no_workloads:
        line["workloads"], checks = workloads_leg(native, torch, stream)
    if args.serve_jobs > 0:
        loads = [float(v) for v in args.serve_loads.split(",") if v]
        line["serving"] = serving_leg(native, torch, args.serve_jobs, loads)
    if not args.no_cpu:
        cb, err = cpu_baseline(x0, w, gpu_out, args.cpu_seconds)
        line["cpu_baseline"] = cb
        line["error_vs_oracle"] = {"normwise_rel_sampled": err, "points": 16}
        if checks:
            errs = check_workloads(checks)
            for name, per in errs.items():
                for eng, e in per.items():
                    if isinstance(e, dict):
                        line["workloads"][name][eng].update(e)
                    else:
                        line["workloads"][name][eng]["error_vs_oracle"] = e
    print(json.dumps(line))


if __name__ == "__main__":
    main()
