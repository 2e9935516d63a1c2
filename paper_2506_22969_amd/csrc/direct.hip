// Direct stencil sweep on the vector ALUs: the same-box baseline for the
// matrix-core engines (FP32, FP64 or bfloat16 hi/lo-plane states).  Each thread produces RY consecutive outputs along y
// of one column, reading each input row segment of its window once.
#include <hip/hip_runtime.h>

#include "kargs.hpp"

namespace ss {

__device__ inline int wrap_i(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Element access of the three state kinds: FP32 and FP64 values as stored;
// planes as hi + lo (exact in FP32), written back as hi = RNE(y),
// lo = RNE(y - hi).
template <int KIND>
struct StateIo;
template <>
struct StateIo<kDirectF32> {
    using T = float;
    __device__ static float load(const void *p, size_t, size_t i) { return static_cast<const float *>(p)[i]; }
    __device__ static void store(void *p, size_t, size_t i, float y) { static_cast<float *>(p)[i] = y; }
};
template <>
struct StateIo<kDirectF64> {
    using T = double;
    __device__ static double load(const void *p, size_t, size_t i) { return static_cast<const double *>(p)[i]; }
    __device__ static void store(void *p, size_t, size_t i, double y) { static_cast<double *>(p)[i] = y; }
};
template <>
struct StateIo<kDirectPlanes> {
    using T = float;
    __device__ static float load(const void *p, size_t plane, size_t i) {
        const __bf16 *b = static_cast<const __bf16 *>(p);
        return (float)b[i] + (float)b[plane + i];
    }
    __device__ static void store(void *p, size_t plane, size_t i, float y) {
        __bf16 *b = static_cast<__bf16 *>(p);
        const __bf16 h = (__bf16)y;
        b[i] = h;
        b[plane + i] = (__bf16)(y - (float)h);
    }
};

template <int KIND, int RAD, int RY>
__global__ __launch_bounds__(256) void k_direct(DirectArgs a) {
    using IO = StateIo<KIND>;
    using T = typename IO::T;
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
    const size_t plane = (size_t)g.nz * g.ny * g.nx;
    const T *w = static_cast<const T *>(a.w);
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
            const size_t row = ((size_t)zz * g.ny + yy) * g.nx;
            T v[2 * RAD + 1];
#pragma unroll
            for (int c = 0; c < 2 * RAD + 1; ++c) {
                v[c] = T(0);
                if (c < kx) {
                    int xx = x - a.rx + c;
                    if (a.periodic) v[c] = IO::load(g.in, plane, row + wrap_i(xx, g.nx));
                    else if (xx >= 0 && xx < g.nx) v[c] = IO::load(g.in, plane, row + xx);
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
        if (y0 + jj < g.ny) IO::store(g.out, plane, ((size_t)z * g.ny + y0 + jj) * g.nx + x, acc[jj]);
}

template <int KIND, int RAD>
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
    hipLaunchKernelGGL((k_direct<KIND, RAD, RY>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int KIND>
static hipError_t launch_r(DirectArgs &a, hipStream_t s) {
    const int r = a.rx;
    if (r <= 1) return launch_t<KIND, 1>(a, s);
    if (r <= 2) return launch_t<KIND, 2>(a, s);
    if (r <= 3) return launch_t<KIND, 3>(a, s);
    if (r <= 6) return launch_t<KIND, 6>(a, s);
    return hipErrorInvalidValue;
}

// Band points of an ny x nx grid within b of an edge: rows 0..b-1, rows
// ny-b..ny-1, then columns 0..b-1 and nx-b..nx-1 of the rows between (the
// whole grid when it is narrower than 2b).
__host__ __device__ inline int band_points(int ny, int nx, int b) {
    if (ny <= 2 * b || nx <= 2 * b) return ny * nx;
    return 2 * b * nx + 2 * b * (ny - 2 * b);
}

// Exact value of two zero-halo sweeps at band point i of a grid:
// y2(p) = sum_a w[a] [p+a in grid] sum_b w[b] x[p+a+b] [p+a+b in grid]
// (correlation, offsets -r..r), in FP64.  The fused launch computed the
// composed stencil on the zero-padded grid, which differs exactly where p+a
// leaves the grid, i.e. within r of an edge.  R > 0: the (4R+1)^2 inputs
// around p are loaded once into registers (zero outside the grid); R = 0:
// any radius, straight from memory.
template <int R>
__global__ __launch_bounds__(256) void k_edge2d(EdgeArgs a) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= a.total) return;
    int j = 0;
    for (int t = 1; t < a.njobs; ++t) j += idx >= a.job[t].point0 ? 1 : 0;
    const EdgeJob &g = a.job[j];
    const int b = R > 0 ? R : a.rad, k = 2 * b + 1;
    int l = idx - g.point0, y, x;
    if (g.ny <= 2 * b || g.nx <= 2 * b) {
        y = l / g.nx;
        x = l % g.nx;
    } else if (l < 2 * b * g.nx) {
        const int r = l / g.nx;
        y = r < b ? r : g.ny - 2 * b + r;
        x = l % g.nx;
    } else {
        l -= 2 * b * g.nx;
        const int r = l / (2 * b), c = l % (2 * b);
        y = b + r;
        x = c < b ? c : g.nx - 2 * b + c;
    }
    double acc = 0.0;
    if constexpr (R > 0) {
        constexpr int E = 4 * R + 1;
        float xs[E][E];
#pragma unroll
        for (int i = 0; i < E; ++i)
#pragma unroll
            for (int c = 0; c < E; ++c) {
                const int sy = y - 2 * R + i, sx = x - 2 * R + c;
                xs[i][c] = (sy >= 0 && sy < g.ny && sx >= 0 && sx < g.nx) ? g.in[(size_t)sy * g.nx + sx] : 0.f;
            }
#pragma unroll
        for (int ay = -R; ay <= R; ++ay)
#pragma unroll
            for (int ax = -R; ax <= R; ++ax) {
                if (y + ay < 0 || y + ay >= g.ny || x + ax < 0 || x + ax >= g.nx) continue;
                double inner = 0.0;
#pragma unroll
                for (int by = -R; by <= R; ++by)
#pragma unroll
                    for (int bx = -R; bx <= R; ++bx)
                        inner += a.w[(by + R) * k + (bx + R)] * (double)xs[2 * R + ay + by][2 * R + ax + bx];
                acc += a.w[(ay + R) * k + (ax + R)] * inner;
            }
    } else {
        for (int ay = -b; ay <= b; ++ay)
            for (int ax = -b; ax <= b; ++ax) {
                const int qy = y + ay, qx = x + ax;
                if (qy < 0 || qy >= g.ny || qx < 0 || qx >= g.nx) continue;
                double inner = 0.0;
                for (int by = -b; by <= b; ++by)
                    for (int bx = -b; bx <= b; ++bx) {
                        const int sy = qy + by, sx = qx + bx;
                        if (sy < 0 || sy >= g.ny || sx < 0 || sx >= g.nx) continue;
                        inner += a.w[(by + b) * k + (bx + b)] * (double)g.in[(size_t)sy * g.nx + sx];
                    }
                acc += a.w[(ay + b) * k + (ax + b)] * inner;
            }
    }
    g.out[(size_t)y * g.nx + x] = (float)acc;
}

hipError_t launch_edge2d(EdgeArgs &a, hipStream_t s) {
    if (a.njobs < 1 || a.njobs > kMaxJobs || a.rad < 1) return hipErrorInvalidValue;
    long long total = 0;
    for (int j = 0; j < a.njobs; ++j) {
        a.job[j].point0 = (int)total;
        total += band_points(a.job[j].ny, a.job[j].nx, a.rad);
    }
    if (total > (1ll << 31) - 256) return hipErrorInvalidValue;
    a.total = (int)total;
    if (total == 0) return hipSuccess;
    const dim3 grid((unsigned)((total + 255) / 256));
    if (a.rad == 1) hipLaunchKernelGGL(k_edge2d<1>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_edge2d<0>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_direct(DirectArgs &a, int kind, hipStream_t s) {
    if (a.njobs < 1 || a.njobs > kMaxJobs) return hipErrorInvalidValue;
    switch (kind) {
        case kDirectF32: return launch_r<kDirectF32>(a, s);
        case kDirectF64: return launch_r<kDirectF64>(a, s);
        case kDirectPlanes: return launch_r<kDirectPlanes>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ss
