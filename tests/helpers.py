"""Shared helpers of the GPU parity tests (oracle side only)."""
from __future__ import annotations

import numpy as np

from oracle import direct  # noqa: F401
from oracle.sampling import cone_sample, sample_points  # noqa: F401

# Bounds stated for results on an FP32 state (normwise relative error after
# all T sweeps): the binary16-split and FP32 paths are held to STATED_F32,
# and to STATED_SPLIT where the path reaches it (fused radius-1 sweeps, the
# 3-D and 1-D workloads).  bfloat16 parts (and the bfloat16 planes state)
# round at 2^-8 per part and are held to their a-priori bound only.
STATED_F32 = 1e-5
STATED_SPLIT = 1e-6
U_BF16 = 2.0 ** -8


def normwise_err(got: np.ndarray, ref: np.ndarray) -> float:
    """max |got - ref| / max |ref| (elementwise relative error is meaningless
    near the zeros mixed-sign stencils produce)."""
    den = float(np.abs(ref).max())
    return float(np.abs(got.astype(np.float64) - ref).max()) / (den if den > 0 else 1.0)


def split_step_bound(fmt: str, n_mma: int) -> float:
    """A-priori relative error of one split-precision sweep, per unit of
    sum|c| * max|x|: the dropped lo*lo product and the roundings of the
    coefficient and state lo parts (one unit each, u^2 with u the part's unit
    roundoff: 2^-11 for binary16's 11 significant bits, 2^-8 for bfloat16's
    8), FP32 rounding once per accumulating MMA, and the FP32 store."""
    u = 2.0 ** -11 if fmt == "f16" else 2.0 ** -8
    return 3 * u * u + (n_mma + 1) * 2.0 ** -24


def apriori_bound(info: dict, w: np.ndarray, steps: int, dtype: str, k_kernel: int = 0) -> float:
    """A-priori normwise bound after `steps` sweeps of a plan (info is the
    plan's info dict, w the unfused coefficients; k_kernel, when given, the
    length of the launched kernel's K order, which the 3-D kernels pad per
    plane beyond the canonical K_pad).

    Per launch: the split bound of the engine's MMA count times sum|c| of the
    coefficients the launch applies (composed for fused launches); the direct
    FP32 engine 2 (P + 1) 2^-24 sum|c| for its P products; the bfloat16
    planes state adds the re-rounding of the result into two planes (u^2).
    Leftover sweeps of a fused plan run unfused, with no larger K."""
    from oracle import tables as T

    if dtype == "f64":
        return 1e-13
    w = np.asarray(w, dtype=np.float64)
    fuse = int(info["fuse_steps"])
    ws = T.compose(w, fuse) if fuse > 1 else w
    eng = info["engine_name"]

    def per_launch(wc):
        s = float(np.abs(wc).sum())
        if eng == "direct":
            b = 2 * (np.count_nonzero(wc) + 1) * 2.0 ** -24 * s
        else:
            fmt = "f16" if dtype == "f32_split_f16" else "bf16"
            chunk = 64 if eng == "smfmac" else 32
            b = split_step_bound(fmt, 3 * max(int(info["k_pad"]), k_kernel) // chunk) * s
        return b + (U_BF16 ** 2 if dtype == "split_bf16" else 0.0)

    return (steps // fuse) * per_launch(ws) + (steps % fuse) * per_launch(w)


def planes_value(bits: np.ndarray) -> np.ndarray:
    """(2, ...) uint16 bfloat16 bit patterns -> hi + lo in FP64."""
    f = (np.asarray(bits).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return f[0] + f[1]
