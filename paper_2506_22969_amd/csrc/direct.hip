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
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * RY;
    const int z = blockIdx.z;
    if (x >= a.nx || y0 >= a.ny) return;
    const T *in = static_cast<const T *>(a.in);
    const T *w = static_cast<const T *>(a.w);
    T *out = static_cast<T *>(a.out);
    const int kz = 2 * a.rz + 1, ky = 2 * a.ry + 1, kx = 2 * a.rx + 1;
    T acc[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) acc[j] = T(0);
    for (int az = 0; az < kz; ++az) {
        int zz = z - a.rz + az;
        if (a.periodic) zz = wrap_i(zz, a.nz);
        else if (zz < 0 || zz >= a.nz) continue;
        for (int yi = 0; yi < RY + 2 * a.ry; ++yi) {
            int yy = y0 - a.ry + yi;
            if (a.periodic) yy = wrap_i(yy, a.ny);
            else if (yy < 0 || yy >= a.ny) continue;
            const T *row = in + ((size_t)zz * a.ny + yy) * a.nx;
            T v[2 * RAD + 1];
#pragma unroll
            for (int c = 0; c < 2 * RAD + 1; ++c) {
                v[c] = T(0);
                if (c < kx) {
                    int xx = x - a.rx + c;
                    if (a.periodic) v[c] = row[wrap_i(xx, a.nx)];
                    else if (xx >= 0 && xx < a.nx) v[c] = row[xx];
                }
            }
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                const int b = yi - j;
                if (b < 0 || b >= ky) continue;
                const T *wr = w + ((size_t)az * ky + b) * kx;
#pragma unroll
                for (int c = 0; c < 2 * RAD + 1; ++c)
                    if (c < kx) acc[j] += wr[c] * v[c];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < RY; ++j)
        if (y0 + j < a.ny) out[((size_t)z * a.ny + y0 + j) * a.nx + x] = acc[j];
}

template <typename T, int RAD>
static hipError_t launch_t(const DirectArgs &a, hipStream_t s) {
    constexpr int RY = 4;
    const int ry_eff = a.ny > 1 ? RY : 1;
    dim3 grid((a.nx + 63) / 64, (a.ny + 4 * ry_eff - 1) / (4 * ry_eff), a.nz);
    if (a.ny > 1)
        hipLaunchKernelGGL((k_direct<T, RAD, RY>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_direct<T, RAD, 1>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_r(const DirectArgs &a, hipStream_t s) {
    const int r = a.rx;
    if (r <= 1) return launch_t<T, 1>(a, s);
    if (r <= 2) return launch_t<T, 2>(a, s);
    if (r <= 3) return launch_t<T, 3>(a, s);
    if (r <= 6) return launch_t<T, 6>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_direct(const DirectArgs &a, int is_f64, hipStream_t s) {
    return is_f64 ? launch_r<double>(a, s) : launch_r<float>(a, s);
}

}  // namespace ss
