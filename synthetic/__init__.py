"""Seeded synthetic inputs for stencil runs.

This module only draws random numbers and lays them out as grids, coefficient
arrays and job streams.  It holds none of the stencil method's arithmetic, so
both the CPU oracle side and the GPU side may take their inputs from it.

Recipe (every draw uses numpy's PCG64 generator):

* grids: seed 0 by default, values uniform in [0, 1) drawn in float64 and then
  rounded once to the state type (float32 uses numpy's round-to-nearest-even
  conversion; bf16 hi/lo planes are produced by bit truncation, which is just
  a way of producing some bf16 numbers whose sum is the intended value);
* coefficients: seed 1 by default, u uniform in [-1, 1) on the stencil's
  points, c = u / sum(u); redrawn with seed+1, seed+2, ... until the stencil is
  von Neumann stable (max |W_hat| <= 1 + 1e-12 on a Fourier lattice of the
  grid, capped per axis), so that values stay bounded over many steps;
* the Heat-2D Jacobi stencil has fixed coefficients 0.5 (centre) and 0.125
  (each of the four neighbours);
* serving job streams: seed 2 by default.

Shapes follow the paper's stencil benchmark table (Section 4.1, Table 1):
star stencils use the centre plus the points on the axes, box stencils every
point of the (2r+1)^d bounding box.
"""
from __future__ import annotations

import numpy as np

GRID_SEED = 0
COEFF_SEED = 1
STREAM_SEED = 2


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# stencil shapes

def stencil_mask(shape: str, radius: int, ndim: int) -> np.ndarray:
    """Boolean (2r+1)^ndim array marking the points of a 'box' or 'star'."""
    k = 2 * radius + 1
    if shape == "box":
        return np.ones((k,) * ndim, dtype=bool)
    if shape == "star":
        m = np.zeros((k,) * ndim, dtype=bool)
        c = (radius,) * ndim
        for ax in range(ndim):
            for d in range(k):
                idx = list(c)
                idx[ax] = d
                m[tuple(idx)] = True
        return m
    raise ValueError(f"unknown shape {shape!r}")


def heat2d_coeffs() -> np.ndarray:
    """Heat-2D 5-point Jacobi: 0.5 at the centre, 0.125 at each neighbour."""
    w = np.zeros((3, 3))
    w[1, 1] = 0.5
    w[0, 1] = w[2, 1] = w[1, 0] = w[1, 2] = 0.125
    return w


def _max_symbol(w: np.ndarray, grid_shape, cap: int) -> float:
    """max over a Fourier lattice of |sum_o w[o] exp(i theta.o)|.

    The lattice has min(N_d, cap) equispaced frequencies per axis; the sum is
    evaluated with an FFT of w placed at offsets o mod n.
    """
    ndim = w.ndim
    r = (w.shape[0] - 1) // 2
    n = [int(min(int(grid_shape[d]), cap)) for d in range(ndim)]
    a = np.zeros(n)
    for o in np.argwhere(w != 0.0):
        a[tuple(int(o[d] - r) % n[d] for d in range(ndim))] += w[tuple(o)]
    return float(np.abs(np.fft.fftn(a)).max())


def random_coeffs(shape: str, radius: int, ndim: int, seed: int = COEFF_SEED,
                  grid_shape=None, max_tries: int = 100000):
    """Random stencil coefficients normalised to sum 1 and von Neumann stable.

    Returns (w, effective_seed) where w is the dense (2r+1)^ndim float64 array
    (zero off the stencil's points).
    """
    mask = stencil_mask(shape, radius, ndim)
    if grid_shape is None:
        grid_shape = (512,) * ndim
    cap = {1: 4096, 2: 512, 3: 64}[ndim]
    for t in range(max_tries):
        g = rng(seed + t)
        u = g.uniform(-1.0, 1.0, size=int(mask.sum()))
        s = u.sum()
        if abs(s) < 1e-3:
            continue
        w = np.zeros(mask.shape)
        w[mask] = u / s
        if _max_symbol(w, grid_shape, cap) <= 1.0 + 1e-12:
            return w, seed + t
    raise RuntimeError("no stable coefficient draw found")


# ----------------------------------------------------------------------------
# grids

def grid_f64(shape, seed: int = GRID_SEED) -> np.ndarray:
    return rng(seed).random(tuple(int(s) for s in shape))


def grid_f32(shape, seed: int = GRID_SEED) -> np.ndarray:
    return grid_f64(shape, seed).astype(np.float32)


def grid_bf16_planes(shape, seed: int = GRID_SEED) -> np.ndarray:
    """Two bf16 planes as uint16 bit patterns, shape (2, *shape): [hi, lo].

    hi holds the top 16 bits of float32(x); lo the top 16 bits of the float32
    remainder.  Any bf16 pair is a valid state; this recipe just makes hi+lo
    close to a uniform[0,1) draw.
    """
    x = grid_f32(shape, seed)
    hi_bits = (x.view(np.uint32) >> 16).astype(np.uint16)
    hi_val = (hi_bits.astype(np.uint32) << 16).view(np.float32)
    rem = (x - hi_val).astype(np.float32)
    lo_bits = (rem.view(np.uint32) >> 16).astype(np.uint16)
    return np.stack([hi_bits, lo_bits])


def grid_bf16_planes3(shape, seed: int = GRID_SEED) -> np.ndarray:
    """Three bf16 planes as uint16 bit patterns, shape (3, *shape): [hi,
    mid, lo], each the top 16 bits of what the planes before it leave of
    float32(x) (so hi + mid + lo = float32(x) exactly for these draws)."""
    x = grid_f32(shape, seed)
    out = []
    rem = x.copy()
    for _ in range(3):
        bits = (rem.view(np.uint32) >> 16).astype(np.uint16)
        val = (bits.astype(np.uint32) << 16).view(np.float32)
        rem = (rem - val).astype(np.float32)
        out.append(bits)
    return np.stack(out)


# ----------------------------------------------------------------------------
# serving stream

def job_stream(n_jobs: int, rate_per_s: float, seed: int = STREAM_SEED,
               kinds=None, steps_range=(10, 200)):
    """Poisson arrivals of stencil jobs.

    Each job is a dict with arrival time (s), kind (a key of ``kinds``), grid
    shape, steps, dtype tag ('f32' or 'split_bf16') and coefficient seed (one
    of 4 per stencil kind, so that jobs sharing a plan exist).
    """
    if kinds is None:
        kinds = {
            "1d5p": dict(shape="box", radius=2, ndim=1, sizes=[(1 << 20,)]),
            "2d5p": dict(shape="star", radius=1, ndim=2,
                         sizes=[(n, n) for n in (1024, 2048, 4096, 8192)]),
            "2d9p": dict(shape="box", radius=1, ndim=2,
                         sizes=[(n, n) for n in (1024, 2048, 4096, 8192)]),
            "2d13p": dict(shape="star", radius=3, ndim=2,
                          sizes=[(n, n) for n in (1024, 2048, 4096, 8192)]),
            "3d7p": dict(shape="star", radius=1, ndim=3,
                         sizes=[(n, n, n) for n in (128, 192, 256, 320, 384)]),
            "3d27p": dict(shape="box", radius=1, ndim=3,
                          sizes=[(n, n, n) for n in (128, 192, 256, 320, 384)]),
        }
    g = rng(seed)
    names = sorted(kinds)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += g.exponential(1.0 / rate_per_s)
        kind = names[int(g.integers(len(names)))]
        spec = kinds[kind]
        size = spec["sizes"][int(g.integers(len(spec["sizes"])))]
        steps = int(g.integers(steps_range[0], steps_range[1] + 1))
        dtype = "f32" if g.random() < 0.5 else "split_bf16"
        cseed = 100 + 4 * names.index(kind) + int(g.integers(4))
        jobs.append(dict(id=j, arrival=t, kind=kind, shape=spec["shape"],
                         radius=spec["radius"], ndim=spec["ndim"], grid=tuple(size),
                         steps=steps, dtype=dtype, coeff_seed=cseed,
                         grid_seed=1000 + j))
    return jobs
