"""Pins of the FP64 direct stepper (oracle/direct.c) against what the
definition of a stencil sweep fixes (paper Section 2.2): brute-force operator
powers, exact rational arithmetic, constant and quadratic fields, periodic
translation invariance, linearity and thread-count independence."""
from fractions import Fraction

import numpy as np
import pytest

import synthetic
from oracle import bruteforce, direct


def setup_module(_m):
    direct.build(force=False)


@pytest.mark.parametrize("dims,radius,periodic", [
    ((23,), 1, False), ((23,), 2, True), ((7, 9), 1, False), ((7, 9), 2, True),
    ((8, 6), 1, True), ((4, 5, 6), 1, False), ((5, 4, 3), 1, True),
])
def test_operator_power_matches_direct(dims, radius, periodic):
    g = synthetic.rng(11)
    k = 2 * radius + 1
    w = g.uniform(-1, 1, size=(k,) * len(dims))
    x = g.random(dims)
    steps = 3
    L = bruteforce.operator_matrix(dims, radius, w, periodic)
    ref = np.linalg.matrix_power(L, steps) @ x.reshape(-1)
    got = direct.run(x, w, steps, periodic=periodic).reshape(-1)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_dyadic_heat2d_is_exact():
    # Heat-2D coefficients (0.5, 0.125) and inputs with 8 fractional bits:
    # every intermediate fits in 53 bits, so FP64 must equal exact arithmetic.
    g = synthetic.rng(3)
    x = g.integers(0, 256, size=(9, 11)) / 256.0
    w = synthetic.heat2d_coeffs()
    for periodic in (False, True):
        exact = bruteforce.exact_run(x, 1, w, periodic, 4)
        got = direct.run(x, w, 4, periodic=periodic)
        for p, v in exact.items():
            assert Fraction(float(got[p])) == v


def test_rounding_error_within_bound():
    # Random FP64 data: error against exact arithmetic is within T*P*2^-53
    # of the absolute-value sum (one rounding per multiply and per add).
    g = synthetic.rng(4)
    x = g.random((6, 7))
    w = g.uniform(-1, 1, size=(3, 3))
    steps = 3
    exact = bruteforce.exact_run(x, 1, w, False, steps)
    got = direct.run(x, w, steps)
    absw = float(np.abs(w).sum())
    bound = steps * 2 * 9 * 2.0 ** -53 * absw ** steps * float(np.abs(x).max()) * 4
    for p, v in exact.items():
        assert abs(float(got[p]) - float(v)) <= bound


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_constant_field(ndim):
    # A constant field kappa maps to (sum c)^T kappa exactly (dyadic data) on a
    # periodic grid, and at points at least T*r from a zero boundary.
    g = synthetic.rng(5)
    k = 3
    w = g.integers(-8, 9, size=(k,) * ndim) / 16.0
    kappa = 0.75
    dims = {1: (40,), 2: (12, 13), 3: (9, 8, 10)}[ndim]
    x = np.full(dims, kappa)
    steps = 3
    want = float(w.sum()) ** steps * kappa
    per = direct.run(x, w, steps, periodic=True)
    assert np.all(per == want)
    zer = direct.run(x, w, steps, periodic=False)
    inner = tuple(slice(steps, n - steps) for n in dims)
    assert np.all(zer[inner] == want)


def quad_field(ny, nx, a, b, c, d, e, h):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    return a * x * x + b * x * y + c * y * y + d * x + e * y + h


def test_laplacian_of_quadratic_is_exact():
    # 5-point Laplacian of a x^2 + b xy + c y^2 + d x + e y + h is 2a + 2c
    # exactly at interior points.
    lap = np.array([[0, 1, 0], [1, -4, 1], [0, 1, 0]], dtype=np.float64)
    a, b, c, d, e, h = 3, -2, 5, 7, -1, 4
    f = quad_field(12, 14, a, b, c, d, e, h)
    got = direct.run(f, lap, 1)
    assert np.all(got[1:-1, 1:-1] == 2 * a + 2 * c)


def test_heat2d_of_quadratic_is_exact():
    # Heat-2D = identity + Laplacian / 8, so it maps f to f + (2a+2c)/8.
    a, b, c, d, e, h = 1, 2, 3, -4, 5, -6
    f = quad_field(10, 12, a, b, c, d, e, h)
    got = direct.run(f, synthetic.heat2d_coeffs(), 1)
    assert np.all(got[1:-1, 1:-1] == f[1:-1, 1:-1] + 0.125 * (2 * a + 2 * c))


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_periodic_translation_invariance(ndim):
    g = synthetic.rng(6)
    dims = {1: (31,), 2: (9, 10), 3: (6, 7, 5)}[ndim]
    w = g.uniform(-1, 1, size=(5,) * ndim)
    x = g.random(dims)
    shift = tuple(range(1, ndim + 1))
    axes = tuple(range(ndim))
    a = np.roll(direct.run(x, w, 2, periodic=True), shift, axis=axes)
    b = direct.run(np.roll(x, shift, axis=axes), w, 2, periodic=True)
    assert np.array_equal(a, b)


def test_linearity():
    g = synthetic.rng(7)
    w = g.uniform(-1, 1, size=(3, 3))
    x, y = g.random((10, 9)), g.random((10, 9))
    lhs = direct.run(2.0 * x + y, w, 3)
    rhs = 2.0 * direct.run(x, w, 3) + direct.run(y, w, 3)
    assert np.max(np.abs(lhs - rhs)) <= 1e-13


def test_thread_count_does_not_change_result():
    g = synthetic.rng(8)
    w = g.uniform(-1, 1, size=(3, 3, 3))
    x = g.random((12, 11, 10))
    a = direct.run(x, w, 2, nthreads=1)
    b = direct.run(x, w, 2, nthreads=4)
    assert np.array_equal(a, b)


def test_star_is_box_with_zeros():
    # A star stencil is the box stencil with zeros off the axes.
    mask = synthetic.stencil_mask("star", 2, 2)
    assert mask.sum() == 9
    g = synthetic.rng(9)
    w = np.where(mask, g.uniform(-1, 1, size=mask.shape), 0.0)
    x = g.random((9, 8))
    L = bruteforce.operator_matrix((9, 8), 2, w, False)
    assert np.max(np.abs(direct.run(x, w, 1).reshape(-1) - L @ x.reshape(-1))) < 1e-14


@pytest.mark.parametrize("shape,periodic", [((37, 41), False), ((37, 41), True),
                                            ((11, 13, 17), False), ((11, 13, 17), True)])
def test_cone_sample_equals_full_run(shape, periodic):
    # dependency-cone sampling against stepping the whole grid
    from oracle.sampling import cone_sample, sample_points, sample_points3
    ndim = len(shape)
    g = np.random.Generator(np.random.PCG64(3))
    w = g.uniform(-1, 1, (3,) * ndim)
    w /= np.abs(w).sum()
    x = g.random(shape)
    steps = 4
    full = direct.run(x, w, steps, periodic=periodic)
    pts = sample_points(*shape, 12, seed=4) if ndim == 2 else sample_points3(*shape, 12, seed=4)
    got = cone_sample(x, w, steps, pts, periodic=periodic)
    want = np.array([full[p] for p in pts])
    assert np.allclose(got, want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n,radius,steps,periodic", [(61, 1, 5, False), (61, 1, 5, True), (70, 2, 6, False),
                                                     (70, 2, 6, True), (53, 3, 4, False), (29, 2, 9, True)])
def test_cone_sample_1d_equals_operator_power(n, radius, steps, periodic):
    # 1-D dependency-cone sampling (the full-size 1-D GPU checks rest on it)
    # against the explicit operator L^T x, which shares no code with the
    # stepper; the points include both ends, where the window is clipped
    # (zero halo) or wrapped (periodic), and reaches longer than the grid
    from oracle.sampling import cone_sample
    g = np.random.Generator(np.random.PCG64(21))
    k = 2 * radius + 1
    w = g.uniform(-1, 1, k)
    w /= np.abs(w).sum()
    x = g.random(n)
    L = bruteforce.operator_matrix((n,), radius, w, periodic)
    full = np.linalg.matrix_power(L, steps) @ x
    pts = [(0,), (1,), (radius,), (n // 2,), (n - 1 - radius,), (n - 2,), (n - 1,)]
    got = cone_sample(x, w, steps, pts, periodic=periodic)
    want = np.array([full[p[0]] for p in pts])
    assert np.max(np.abs(got - want)) <= 1e-13


def test_binary16_rounding_is_exact_rne():
    """The binary16 oracle rounds with numpy's float64 -> float16 conversion:
    pinned against exact rational round-to-nearest-even on random values,
    exact ties (odd and even neighbours), subnormals and values near the
    largest finite number."""
    from oracle import fpformat
    rng = np.random.default_rng(3)
    vals = list(rng.uniform(-4, 4, 2000)) + list(rng.uniform(-1e-6, 1e-6, 500))
    # ties halfway between binary16 neighbours around 1 (spacing 2^-10)
    vals += [1.0 + (2 * i + 1) * 2.0 ** -11 for i in range(64)]
    vals += [-(1.0 + (2 * i + 1) * 2.0 ** -11) for i in range(64)]
    vals += [(2 * i + 1) * 2.0 ** -25 for i in range(32)]          # subnormal ties
    vals += [65504.0, 65519.0, -65504.0, 6.1e-5, 5.96e-8, 0.0]
    for v in vals:
        ref = fpformat.round_rne(float(v), fpformat.BINARY16)
        assert ref is not None
        assert float(np.float16(v)) == ref, v


def _binary16_bruteforce(x, w, steps):
    """Pure-Python binary16 sweeps on a tiny zero-halo 2-D grid: exact
    rational sums of the rounded coefficients times the rounded state,
    rounded once per sweep."""
    from fractions import Fraction

    from oracle import fpformat
    k = w.shape[0]
    r = k // 2
    ny, nx = x.shape
    wr = [[Fraction(fpformat.round_rne(float(w[a, b]), fpformat.BINARY16)) for b in range(k)] for a in range(k)]
    cur = [[Fraction(fpformat.round_rne(float(x[i, j]), fpformat.BINARY16)) for j in range(nx)] for i in range(ny)]
    for _ in range(steps):
        nxt = []
        for i in range(ny):
            row = []
            for j in range(nx):
                s = Fraction(0)
                for a in range(k):
                    for b in range(k):
                        ii, jj = i - r + a, j - r + b
                        if 0 <= ii < ny and 0 <= jj < nx:
                            s += wr[a][b] * cur[ii][jj]
                row.append(Fraction(fpformat.round_rne(float(s), fpformat.BINARY16)))
            nxt.append(row)
        cur = nxt
    return np.array([[float(v) for v in row] for row in cur])


@pytest.mark.parametrize("radius,steps", [(1, 3), (2, 2)])
def test_binary16_run_equals_bruteforce(radius, steps):
    """run_binary16 against exact rational arithmetic on a tiny grid.  The
    oracle forms each sum in FP64, exact for these few binary16 products up
    to one FP64 rounding, which can decide a binary16 tie only with
    probability ~2^-42; the seeds here hit none."""
    rng = np.random.default_rng(11 + radius)
    k = 2 * radius + 1
    w = rng.uniform(-1, 1, (k, k))
    w /= w.sum()
    x = rng.uniform(0, 1, (6, 7))
    got = direct.run_binary16(x, w, steps)
    ref = _binary16_bruteforce(x, w, steps)
    assert np.array_equal(got, ref)


def test_binary16_constant_field():
    """Heat-2D coefficients and 0.75 are binary16 numbers and every partial
    sum is exact: interior points stay 0.75."""
    w = np.array([[0, 0.125, 0], [0.125, 0.5, 0.125], [0, 0.125, 0]])
    x = np.full((20, 24), 0.75)
    got = direct.run_binary16(x, w, 4)
    assert np.all(got[4:-4, 4:-4] == 0.75)


@pytest.mark.parametrize("periodic", [False, True])
def test_binary16_cone_sample_equals_full_run(periodic):
    """Dependency-cone sampling of the binary16 sweeps (rounding acts point
    by point, so a point's cone still fixes it) against the whole grid."""
    from oracle.sampling import cone_sample, sample_points
    g = np.random.Generator(np.random.PCG64(8))
    w = g.uniform(-1, 1, (3, 3))
    w /= np.abs(w).sum()
    x = g.random((33, 40))
    steps = 5
    full = direct.run_binary16(x, w, steps, periodic=periodic)
    pts = sample_points(33, 40, 14, seed=9)
    got = cone_sample(x, w, steps, pts, periodic=periodic, binary16=True)
    assert np.array_equal(got, np.array([full[p] for p in pts]))
