/*
 * Oracle: plain FP64 stencil stepper.  TEST INFRASTRUCTURE ONLY -- the product
 * path never links or calls this file.
 *
 * It computes the plain definition of an iterated stencil (paper, Section 2.2,
 * and the commented Box-2D9P pseudo-code there): every point of the grid is
 * replaced by the weighted sum of the input points in its (2r+1)^d bounding
 * box, in correlation orientation (coefficient w[a][b] multiplies
 * x[i - r + a][j - r + b]); the result goes to a second mesh and the two meshes
 * swap roles for the next step.
 *
 *   boundary 0: zero halo  -- points outside the domain read as 0
 *   boundary 1: periodic   -- indices wrap modulo the grid size
 *
 * Each point's sum runs over the bounding box in row-major order (slowest
 * dimension first), so the result does not depend on the thread count.
 * Build with -O3 -ffp-contract=off so that no multiply-add gets fused.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline int64_t wrap(int64_t i, int64_t n) {
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

/* one sweep: dst <- W * src on a 3-D grid (nz, ny, nx); radii per axis. */
static void sweep(const double *src, double *dst, int64_t nz, int64_t ny, int64_t nx,
                  int rz, int ry, int rx, const double *w, int periodic) {
    const int kz = 2 * rz + 1, ky = 2 * ry + 1, kx = 2 * rx + 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t x = 0; x < nx; ++x) {
                double acc = 0.0;
                for (int a = 0; a < kz; ++a) {
                    int64_t zz = z - rz + a;
                    if (periodic) zz = wrap(zz, nz);
                    else if (zz < 0 || zz >= nz) continue;
                    for (int b = 0; b < ky; ++b) {
                        int64_t yy = y - ry + b;
                        if (periodic) yy = wrap(yy, ny);
                        else if (yy < 0 || yy >= ny) continue;
                        for (int c = 0; c < kx; ++c) {
                            int64_t xx = x - rx + c;
                            if (periodic) xx = wrap(xx, nx);
                            else if (xx < 0 || xx >= nx) continue;
                            acc += w[(a * ky + b) * kx + c] * src[(zz * ny + yy) * nx + xx];
                        }
                    }
                }
                dst[(z * ny + y) * nx + x] = acc;
            }
        }
    }
}

/*
 * Run `steps` sweeps in place on x (row-major, slowest dimension first).
 * ndim in {1,2,3}; dims[ndim]; w has (2r+1)^ndim entries in the same order.
 * scratch must hold as many doubles as x.  Returns 0, or -1 on bad arguments.
 */
int oracle_direct_run(int ndim, const int64_t *dims, int radius, const double *w,
                      int periodic, int64_t steps, double *x, double *scratch,
                      int nthreads) {
    if (ndim < 1 || ndim > 3 || radius < 0 || steps < 0 || !x || !scratch || !w) return -1;
    int64_t n[3] = {1, 1, 1};
    int r[3] = {0, 0, 0};
    for (int d = 0; d < ndim; ++d) {
        if (dims[d] <= 0) return -1;
        n[3 - ndim + d] = dims[d];
        r[3 - ndim + d] = radius;
    }
#ifdef _OPENMP
    /* a thread count asked for holds for this call only */
    const int prev_threads = omp_get_max_threads();
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    double *a = x, *b = scratch;
    for (int64_t t = 0; t < steps; ++t) {
        sweep(a, b, n[0], n[1], n[2], r[0], r[1], r[2], w, periodic);
        double *tmp = a; a = b; b = tmp;
    }
    if (a != x) memcpy(x, a, (size_t)(n[0] * n[1] * n[2]) * sizeof(double));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(prev_threads);
#endif
    return 0;
}

/* number of OpenMP threads a parallel region would use */
int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
