"""Benchmark: Box-2D9P on a 10240 x 10240 FP32 grid, 100 sweeps, zero halo,
binary16 hi+lo split products on gfx950 sparse MFMA (SMFMAC).

One step = one sparstencil_run of the whole workload (100 sweeps) on grids
already resident in HBM.  Prints one JSON line with GStencil/s (paper
Section 4.1, Eq. 12: T * prod(N_i) / (t * 1e9)), latency percentiles, the
dense-MFMA and direct-FMA engines on the same workload, the roofline of the
sparse sweep kernel (HIP events on its stream) and the CPU oracle baseline.
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
KERNEL_SRC = os.path.join(ROOT, "paper_2506_22969_amd", "csrc", "mma2d.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--engines", default="smfmac,mfma,direct",
                    help="engines to time; the first is the headline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--sweep-loop", type=int, default=40, help="sweeps timed for the roofline")
    return ap.parse_args()


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_entry():
    """Measured HBM bytes per launch, only if taken on the current kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def time_engine(native, torch, w, x0_dev, engine, steps, warmup, stream):
    plan = native.Plan("box", 1, w, (NY, NX), "f32_split_f16", engine=engine)
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


def cpu_baseline(x0: np.ndarray, w: np.ndarray, gpu_out: np.ndarray, budget_s: float):
    """The FP64 oracle on the host cores: full-grid sweeps for about budget_s
    seconds (throughput), then sampled outputs of the 100-sweep run through
    their dependency cones (error of the GPU result)."""
    from oracle import direct as oracle_direct
    from oracle.sampling import cone_sample, sample_points

    xd = x0.astype(np.float64)
    t0 = time.perf_counter()
    oracle_direct.run(xd, w, 1)
    t1 = time.perf_counter() - t0
    n = max(1, int(budget_s / max(t1, 1e-3)))
    t0 = time.perf_counter()
    oracle_direct.run(xd, w, n)
    dt = time.perf_counter() - t0
    pts = sample_points(NY, NX, 16, seed=1)
    ref = cone_sample(x0, w, SWEEPS, pts)
    vals = np.array([gpu_out[y, x] for (y, x) in pts], dtype=np.float64)
    err = float(np.abs(vals - ref).max() / np.abs(ref).max())
    return {"value": n * NY * NX / dt / 1e9, "unit": "GStencil/s", "cores": oracle_direct.threads(),
            "kind": "oracle",
            "sample": f"{n} full-grid FP64 sweeps of the 10240^2 Box-2D9P grid ({dt:.1f} s); "
                      f"error check on 16 sampled outputs of the 100-sweep run via dependency cones"}, err


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
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
    for i, eng in enumerate(engines):
        steps = args.steps if i == 0 else max(2, args.steps // 3)
        plan, info, lat, t_total, out = time_engine(native, torch, w, x0_dev, eng, steps, args.warmup, stream)
        gst = SWEEPS * NY * NX / (t_total / steps) / 1e9
        results[eng] = {"gstencil_s": round(gst, 2), "ms_per_run": round(t_total / steps * 1e3, 3),
                        "tile": [info["r1"], info["r2"]], "k_pad": info["k_pad"],
                        "plan_ms": round(info["plan_seconds"] * 1e3, 3)}
        if i == 0:
            head = (plan, info, lat, t_total, steps, out.cpu().numpy())
        else:
            plan.close()
        sys.stdout.flush()
    plan, info, lat, t_total, steps, gpu_out = head
    ms = t_total / steps * 1e3
    value = SWEEPS * NY * NX / (ms / 1e3) / 1e9

    sweep_ms = sweep_roofline(torch, plan, x0_dev, stream, args.sweep_loop)
    alg_bytes = BYTES_PER_POINT * NY * NX
    achieved = alg_bytes / (sweep_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_entry(),
            "kernel": "k_mma2d (sparse, binary16 split)", "sweep_ms": round(sweep_ms, 4),
            "algorithmic_bytes_per_launch": alg_bytes}
    plan.close()

    line = {
        "metric": "GStencil/s + % HBM/SMFMAC peak vs dense-MFMA/direct at stated error; p99 lat",
        "value": round(value, 2), "unit": "GStencil/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "Box-2D9P 10240x10240 FP32 state, binary16 hi+lo split products "
                               "with FP32 accumulation, 100 sweeps, zero halo",
                   "engine": engines[0], "tile": [info["r1"], info["r2"]], "k_pad": info["k_pad"],
                   "coeff_seed": cseed, "grid_seed": 0, "accumulate": "f32"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3)},
        "engines": results,
        "roofline": roof,
    }
    if not args.no_cpu:
        cb, err = cpu_baseline(x0, w, gpu_out, args.cpu_seconds)
        line["cpu_baseline"] = cb
        line["error_vs_oracle"] = {"normwise_rel_sampled": err, "points": 16}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
