"""The kernels' A operand registers against the oracle, on the CPU: each
plan's fragments (SS_Q_KERNEL_FRAGS) decoded with the measured operand
layout (tests/mma_model.py) must be, bit for bit, the oracle's split A' in
the kernel's K order -- for staircase layouts, the re-paired layouts of
stencils with unused columns (Section 3.2's general matcher), custom point
patterns, fused stencils, 1-D and 3-D plans.  Then one sweep of a small grid
through the decoded operands (patches gathered by the K order) matches the
FP64 oracle within the split bound: the tables and the layout model
together compute the stencil."""
import numpy as np
import pytest

import synthetic
from oracle import direct as oracle_direct
from oracle import tables as T

from .mma_model import bits_value, decode

native = pytest.importorskip("paper_2506_22969_amd.native")

SIGMA = {"f16": 2048.0, "bf16": 1.0}

CASES = [  # (ndim, shape, radius, fuse, dtype, engine, tile, seed)
    (2, "box", 1, 1, "f32_split_f16", "smfmac", (8, 8), 1),
    (2, "box", 1, 3, "f32_split_f16", "smfmac", (8, 8), 1),
    (2, "box", 1, 3, "f32_split_f16", "smfmac", (8, 2), 1),
    (2, "star", 3, 1, "f32_split_bf16", "smfmac", (8, 4), 45),
    (2, "star", 1, 3, "f32_split_f16", "smfmac", (0, 0), 45),
    (2, "star", 3, 2, "split_bf16", "smfmac", (8, 4), 45),
    (2, "box", 3, 2, "split3_bf16", "smfmac", (8, 2), 277),
    (2, "star", 1, 1, "f32_split_f16", "mfma", (8, 8), 1),
    (2, "box", 3, 1, "f32_split_bf16", "mfma", (0, 0), 277),
    (1, "box", 3, 2, "f32_split_f16", "smfmac", (16, 1), 3),
    (1, "box", 2, 3, "f32_split_f16", "smfmac", (16, 1), 3),
    (1, "box", 1, 1, "f32_split_f16", "mfma", (16, 1), 3),
    (3, "star", 1, 2, "f32_split_f16", "smfmac", (8, 2), 29),
    (3, "box", 1, 1, "f32_split_f16", "smfmac", (8, 4), 70),
    (3, "box", 1, 2, "f32_split_bf16", "mfma", (8, 2), 70),
]


def _plan(ndim, shape, radius, fuse, dtype, engine, tile, seed):
    dims = {1: (5000,), 2: (256, 256), 3: (24, 48, 264)}[ndim]
    gs = {1: (4096,), 2: dims, 3: None}[ndim]
    w = synthetic.random_coeffs(shape, radius, ndim, seed=seed, grid_shape=gs)[0]
    kw = dict(boundary="periodic", fuse_steps=fuse) if fuse > 1 else {}
    r1, r2 = tile
    if ndim != 2:
        r1 = r2 = 0
    return w, native.Plan(shape, radius, w, dims, dtype, engine=engine, r1=r1, r2=r2, host_only=True, **kw)


def _oracle_parts(a, perm, dtype):
    cols = np.where(perm >= 0, perm, 0)
    ap = np.where(perm[None, :] >= 0, a[:, cols], 0.0)
    if dtype == "split3_bf16":
        return dict(zip(("hi", "mid", "lo"), T.split_three_bf16(ap))), "bf16"
    fmt = "f16" if dtype == "f32_split_f16" else "bf16"
    hi, lo = T.split_hilo(ap, fmt)
    return {"hi": hi, "lo": lo}, fmt


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(str(v) for v in c[:6]))
def test_fragments_are_the_oracle_matrix(case):
    ndim = case[0]
    w, p = _plan(*case)
    with p:
        info = p.info
        fr = p.kernel_fragments()
        perm = p.table(native.Q_KERNEL_PERM)
        wk = p.table(native.Q_COEFFS).reshape((info["k"],) * ndim)
    assert fr["mode"] == ("sparse" if case[5] == "smfmac" else "dense")
    dense, clashes = decode(fr)
    assert clashes == []
    a, _, _ = T.morph(wk, info["r1"], info["r2"])
    want, _ = _oracle_parts(a, perm, case[4])
    for part, bits in want.items():
        got = dense[part][: a.shape[0], : len(perm)]
        assert got.shape == bits.shape
        bad = np.argwhere(got != bits)
        assert bad.size == 0, (part, bad[:5])


@pytest.mark.parametrize("case", [c for c in CASES if c[0] == 2 and c[4].startswith("f32")],
                         ids=lambda c: "-".join(str(v) for v in c[:6]))
def test_decoded_operands_sweep_like_the_oracle(case):
    """One sweep of a small periodic grid: every r2 x r1 tile's patch
    gathered in the kernel's K order (B), multiplied by the decoded A parts
    the way the split products are (hi*hi + (hi*lo + lo*hi) / sigma, with
    the state split the same way), against the FP64 oracle."""
    w, p = _plan(*case)
    with p:
        info = p.info
        fr = p.kernel_fragments()
        perm = p.table(native.Q_KERNEL_PERM)
        wk = p.table(native.Q_COEFFS).reshape(info["k"], info["k"])
    dense, _ = decode(fr)
    parts, fmt = _oracle_parts(np.zeros((1, 1)), np.zeros(0, dtype=np.int32), case[4])
    sig = SIGMA[fmt]
    ahi = bits_value(dense["hi"], fmt)[:, : len(perm)]
    alo = bits_value(dense["lo"], fmt)[:, : len(perm)]
    r1, r2, k = info["r1"], info["r2"], info["k"]
    rad = (k - 1) // 2
    d = T.morph_dims(k, r1, r2, 2)
    ny, nx = 2 * r2 * 2, 3 * r1
    x = synthetic.grid_f32((ny, nx), seed=5).astype(np.float64)
    xh, xl = T.split_hilo(x, fmt)
    xhv, xlv = bits_value(xh, fmt), bits_value(xl, fmt)
    y = np.zeros((ny, nx))
    for ty0 in range(0, ny, r2):
        for tx0 in range(0, nx, r1):
            bh = np.zeros(len(perm))
            bl = np.zeros(len(perm))
            for kk, col in enumerate(perm):
                if col < 0:
                    continue
                pr, pc = (col % (d.m_b * d.g)) // d.g, col % d.g
                yy, xx = (ty0 - rad + pr) % ny, (tx0 - rad + pc) % nx
                bh[kk], bl[kk] = xhv[yy, xx], xlv[yy, xx]
            out = ahi @ bh + (ahi @ bl + alo @ bh) / sig
            for t in range(r1 * r2):
                y[ty0 + t // r1, tx0 + t % r1] = out[t]
    ref = oracle_direct.run(x, np.asarray(wk, dtype=np.float64), 1, periodic=True)
    u = 2.0 ** -11 if fmt == "f16" else 2.0 ** -8
    tol = 3 * u * u * float(np.abs(wk).sum()) * float(np.abs(x).max()) * 4
    assert np.abs(y - ref).max() <= tol
