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
