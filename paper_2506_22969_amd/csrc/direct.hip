// Direct stencil sweep on the vector ALUs: the same-box baseline for the
// matrix-core engines.  Each thread produces RY consecutive outputs along y
// of one column, reading each input row segment of its window once.
#include <hip/hip_runtime.h>

#include "kargs.hpp"

namespace ss {

__device__ inline int wrap_i(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

template <typename T, int RAD, int RY>
__global__ __launch_bounds__(256) void k_direct(DirectArgs a) {
    // block -> (job, z, row block, column block)
    const int b = blockIdx.x;
    int j = 0;
    for (int t = 1; t < a.njobs; ++t) j += b >= a.job[t].block0 ? 1 : 0;
    const DirectJob &g = a.job[j];
    const int nbx = (g.nx + 63) / 64, nby = (g.ny + 4 * RY - 1) / (4 * RY);
    int local = b - g.block0;
    const int bx = local % nbx;
    local /= nbx;
    const int by = local % nby;
    const int z = local / nby;
    const int x = bx * 64 + (threadIdx.x & 63);
    const int y0 = (by * 4 + (threadIdx.x >> 6)) * RY;
    if (x >= g.nx || y0 >= g.ny) return;
    const T *in = static_cast<const T *>(g.in);
    const T *w = static_cast<const T *>(a.w);
    T *out = static_cast<T *>(g.out);
    const int kz = 2 * a.rz + 1, ky = 2 * a.ry + 1, kx = 2 * a.rx + 1;
    T acc[RY];
#pragma unroll
    for (int jj = 0; jj < RY; ++jj) acc[jj] = T(0);
    for (int az = 0; az < kz; ++az) {
        int zz = z - a.rz + az;
        if (a.periodic) zz = wrap_i(zz, g.nz);
        else if (zz < 0 || zz >= g.nz) continue;
        for (int yi = 0; yi < RY + 2 * a.ry; ++yi) {
            int yy = y0 - a.ry + yi;
            if (a.periodic) yy = wrap_i(yy, g.ny);
            else if (yy < 0 || yy >= g.ny) continue;
            const T *row = in + ((size_t)zz * g.ny + yy) * g.nx;
            T v[2 * RAD + 1];
#pragma unroll
            for (int c = 0; c < 2 * RAD + 1; ++c) {
                v[c] = T(0);
                if (c < kx) {
                    int xx = x - a.rx + c;
                    if (a.periodic) v[c] = row[wrap_i(xx, g.nx)];
                    else if (xx >= 0 && xx < g.nx) v[c] = row[xx];
                }
            }
#pragma unroll
            for (int jj = 0; jj < RY; ++jj) {
                const int bb = yi - jj;
                if (bb < 0 || bb >= ky) continue;
                const T *wr = w + ((size_t)az * ky + bb) * kx;
#pragma unroll
                for (int c = 0; c < 2 * RAD + 1; ++c)
                    if (c < kx) acc[jj] += wr[c] * v[c];
            }
        }
    }
#pragma unroll
    for (int jj = 0; jj < RY; ++jj)
        if (y0 + jj < g.ny) out[((size_t)z * g.ny + y0 + jj) * g.nx + x] = acc[jj];
}

template <typename T, int RAD>
static hipError_t launch_t(DirectArgs &a, hipStream_t s) {
    constexpr int RY = 4;
    int blocks = 0;
    for (int j = 0; j < a.njobs; ++j) {
        const DirectJob &g = a.job[j];
        a.job[j].block0 = blocks;
        blocks += ((g.nx + 63) / 64) * ((g.ny + 4 * RY - 1) / (4 * RY)) * g.nz;
    }
    a.total_blocks = blocks;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_direct<T, RAD, RY>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_r(DirectArgs &a, hipStream_t s) {
    const int r = a.rx;
    if (r <= 1) return launch_t<T, 1>(a, s);
    if (r <= 2) return launch_t<T, 2>(a, s);
    if (r <= 3) return launch_t<T, 3>(a, s);
    if (r <= 6) return launch_t<T, 6>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_direct(DirectArgs &a, int is_f64, hipStream_t s) {
    if (a.njobs < 1 || a.njobs > kMaxJobs) return hipErrorInvalidValue;
    return is_f64 ? launch_r<double>(a, s) : launch_r<float>(a, s);
}

}  // namespace ss
