"""Shared helpers of the GPU parity tests (oracle side only)."""
from __future__ import annotations

import numpy as np

from oracle import direct  # noqa: F401
from oracle.sampling import cone_sample, sample_points  # noqa: F401


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
