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
    static_assert(kDirectMaxRad == 6, "widest instantiated radius");
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

// Band point i of a launch -> its grid and (y, x), band width b.
__device__ inline const EdgeJob &band_point(const EdgeArgs &a, int idx, int b, int *py, int *px) {
    int j = 0;
    for (int t = 1; t < a.njobs; ++t) j += idx >= a.job[t].point0 ? 1 : 0;
    const EdgeJob &g = a.job[j];
    int l = idx - g.point0;
    if (g.ny <= 2 * b || g.nx <= 2 * b) {
        *py = l / g.nx;
        *px = l % g.nx;
    } else if (l < 2 * b * g.nx) {
        const int r = l / g.nx;
        *py = r < b ? r : g.ny - 2 * b + r;
        *px = l % g.nx;
    } else {
        l -= 2 * b * g.nx;
        const int r = l / (2 * b), c = l % (2 * b);
        *py = b + r;
        *px = c < b ? c : g.nx - 2 * b + c;
    }
    return g;
}

// Exact value of S zero-halo sweeps at a band point p: y_s = W y_{s-1} with
// every intermediate state zero outside the grid (correlation, offsets
// -r..r), in FP64.  The fused launch applied the composed stencil to the
// zero-padded grid, which differs exactly where an intermediate point p+a
// leaves the grid, i.e. within r(S-1) of an edge.  R > 0: the inputs within
// RS of p are loaded once into registers and each sweep is evaluated on the
// shrinking square of points it still feeds; R = 0 (two sweeps of any
// radius): straight from memory.
template <int R, int S>
__global__ __launch_bounds__(256) void k_edge2d(EdgeArgs a) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= a.total) return;
    const int b = R > 0 ? R * (S - 1) : a.rad;
    int y, x;
    const EdgeJob &g = band_point(a, idx, b, &y, &x);
    double result = 0.0;
    if constexpr (R > 0) {
        constexpr int K = 2 * R + 1;
        constexpr int H = R * S;            // half width of the input square
        constexpr int E = 2 * H + 1;
        double cur[E][E];
        // branch-free: every load is issued (at a clamped address) and
        // out-of-grid values are selected away, so the loads overlap
#pragma unroll
        for (int i = 0; i < E; ++i)
#pragma unroll
            for (int c = 0; c < E; ++c) {
                const int sy = y - H + i, sx = x - H + c;
                const int cy = min(max(sy, 0), g.ny - 1), cx = min(max(sx, 0), g.nx - 1);
                const float v = g.in[(size_t)cy * g.nx + cx];
                cur[i][c] = (sy >= 0 && sy < g.ny && sx >= 0 && sx < g.nx) ? (double)v : 0.0;
            }
        double w[K][K];
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int c = 0; c < K; ++c) w[i][c] = a.w[i * K + c];
        // sweep s maps the square of half width H - (s-1)R to H - sR
#pragma unroll
        for (int s = 1; s <= S; ++s) {
            const int h = H - s * R;        // half width after sweep s
#pragma unroll
            for (int i = 0; i < E; ++i)
#pragma unroll
                for (int c = 0; c < E; ++c) {
                    if (i < H - h || i > H + h || c < H - h || c > H + h) continue;
                    const int sy = y - H + i, sx = x - H + c;
                    double v = 0.0;
#pragma unroll
                    for (int dy = 0; dy < K; ++dy)
#pragma unroll
                        for (int dx = 0; dx < K; ++dx) v += w[dy][dx] * cur[i - R + dy][c - R + dx];
                    v = (sy >= 0 && sy < g.ny && sx >= 0 && sx < g.nx) ? v : 0.0;
                    // written in place from the outside in is unsafe, so
                    // results of this sweep go to the corner block first
                    cur[i - (H - h)][c - (H - h)] = v;
                }
            // move the new square (stored at the top-left) back to the centre
#pragma unroll
            for (int i = E - 1; i >= 0; --i)
#pragma unroll
                for (int c = E - 1; c >= 0; --c) {
                    if (i < H - h || i > H + h || c < H - h || c > H + h) continue;
                    cur[i][c] = cur[i - (H - h)][c - (H - h)];
                }
        }
        result = cur[H][H];
    } else {
        const int k = 2 * b + 1;
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
                result += a.w[(ay + b) * k + (ax + b)] * inner;
            }
    }
    g.out[(size_t)y * g.nx + x] = (float)result;
}

hipError_t launch_edge2d(EdgeArgs &a, hipStream_t s) {
    if (a.njobs < 1 || a.njobs > kMaxJobs || a.rad < 1 || a.steps < 2 || a.steps > 3) return hipErrorInvalidValue;
    if (a.steps == 3 && a.rad != 1) return hipErrorInvalidValue;
    const int b = a.rad * (a.steps - 1);
    long long total = 0;
    for (int j = 0; j < a.njobs; ++j) {
        a.job[j].point0 = (int)total;
        total += band_points(a.job[j].ny, a.job[j].nx, b);
    }
    if (total > (1ll << 31) - 256) return hipErrorInvalidValue;
    a.total = (int)total;
    if (total == 0) return hipSuccess;
    const dim3 grid((unsigned)((total + 255) / 256));
    if (a.rad == 1 && a.steps == 2) hipLaunchKernelGGL((k_edge2d<1, 2>), grid, dim3(256), 0, s, a);
    else if (a.rad == 1) hipLaunchKernelGGL((k_edge2d<1, 3>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_edge2d<0, 2>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// Several sweeps of a small 2-D FP64 grid in one launch (temporal
// blocking): each workgroup owns a kTbTile x kTbTile output tile, loads the
// inputs within H = S*r of it into LDS (zero outside a zero-halo grid,
// wrapped on a periodic one), applies the S sweeps there -- sweep s on the
// window shrunk by s*r from each side, the part the later sweeps still read,
// with points outside a zero-halo grid held at zero -- and stores its tile.
// Each point's sum runs in k_direct's order (rows, then columns, fused
// multiply-adds; the zeros of a zero halo add nothing), so the result is
// bit for bit that of S single-sweep launches.
// Compute units and XCDs of the current device (defined with the 2-D
// matrix kernels' launch code).
hipError_t device_shape(int *cus, int *xcds);

// The tile is 32 x 32, or 16 x 16 when 32 x 32 tiles would leave most
// compute units idle.
template <int RAD, int TILE>
__global__ __launch_bounds__(256) void k_tb2d(DirectArgs a) {
    constexpr int WIN = TILE + 2 * kTbHalo;
    __shared__ double buf[2][WIN * WIN];
    const DirectJob &g = a.job[0];
    const int S = a.steps, H = S * RAD, W = TILE + 2 * H;
    const int ntx = (g.nx + TILE - 1) / TILE;
    const int y0 = (int)(blockIdx.x / ntx) * TILE - H, x0 = (int)(blockIdx.x % ntx) * TILE - H;
    const double *in = static_cast<const double *>(g.in);
    const double *w = static_cast<const double *>(a.w);
    for (int i = threadIdx.x; i < W * W; i += 256) {
        int gy = y0 + i / W, gx = x0 + i % W;
        double v = 0.0;
        if (a.periodic) {
            gy = wrap_i(gy, g.ny);
            gx = wrap_i(gx, g.nx);
            v = in[(size_t)gy * g.nx + gx];
        } else if (gy >= 0 && gy < g.ny && gx >= 0 && gx < g.nx) {
            v = in[(size_t)gy * g.nx + gx];
        }
        buf[0][i] = v;
    }
    __syncthreads();
    for (int st = 1; st <= S; ++st) {
        const double *src = buf[(st - 1) & 1];
        double *dst = buf[st & 1];
        const int lo = st * RAD, n = W - 2 * lo;
        for (int i = threadIdx.x; i < n * n; i += 256) {
            const int wy = lo + i / n, wx = lo + i % n;
            const int gy = y0 + wy, gx = x0 + wx;
            double acc = 0.0;
            if (a.periodic || (gy >= 0 && gy < g.ny && gx >= 0 && gx < g.nx)) {
#pragma unroll
                for (int dy = 0; dy < 2 * RAD + 1; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 2 * RAD + 1; ++dx)
                        acc = __builtin_fma(w[dy * (2 * RAD + 1) + dx], src[(wy - RAD + dy) * W + wx - RAD + dx], acc);
            }
            dst[wy * W + wx] = acc;
        }
        __syncthreads();
    }
    const double *res = buf[S & 1];
    double *out = static_cast<double *>(g.out);
    for (int i = threadIdx.x; i < TILE * TILE; i += 256) {
        const int wy = H + i / TILE, wx = H + i % TILE;
        const int gy = y0 + wy, gx = x0 + wx;
        if (gy < g.ny && gx < g.nx) out[(size_t)gy * g.nx + gx] = res[wy * W + wx];
    }
}

hipError_t launch_direct_tb(DirectArgs &a, hipStream_t s) {
    if (a.njobs != 1 || a.steps < 1 || a.steps * a.rx > kTbHalo || a.rx != a.ry || a.rz != 0)
        return hipErrorInvalidValue;
    const DirectJob &g = a.job[0];
    int cus = 0, xcds = 0;
    if (const hipError_t e = device_shape(&cus, &xcds); e != hipSuccess) return e;
    const int big = ((g.nx + 31) / 32) * ((g.ny + 31) / 32);
    const bool small = big < cus;
    const int t = small ? 16 : 32;
    const int blocks = ((g.nx + t - 1) / t) * ((g.ny + t - 1) / t);
#define SS_TB(R)                                                                                  \
    case R:                                                                                       \
        if (small) hipLaunchKernelGGL((k_tb2d<R, 16>), dim3(blocks), dim3(256), 0, s, a);         \
        else hipLaunchKernelGGL((k_tb2d<R, 32>), dim3(blocks), dim3(256), 0, s, a);              \
        break;
    switch (a.rx) {
        SS_TB(1)
        SS_TB(2)
        SS_TB(3)
        SS_TB(4)
        default: return hipErrorInvalidValue;
    }
#undef SS_TB
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
