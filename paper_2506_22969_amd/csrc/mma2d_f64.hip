// 2-D stencil sweep as a dense FP64 matrix product on gfx950 matrix cores
// (v_mfma_f64_16x16x4_f64): the FP64 baseline of the paper's FP64 study
// (Section 4.7), with the staircase matrix A' of Section 3.1 in FP64 and no
// split.  Tiles of 8 x 4 outputs; a workgroup of 4 waves computes a
// 128 x 16 block from an FP64 slab in LDS (block plus halo, loaded with
// plain loads: the FP64 workloads here are small and launch-bound).
//
// Operand layouts (gfx950, measured): A lane l holds row l%16, K = l/16; B
// lane l holds column l%16, K = l/16; accumulator lane l holds column l%16,
// rows 4*i + l/16 (i = 0..3).
#include <hip/hip_runtime.h>

#include "kargs.hpp"
#include "kgeom.hpp"

namespace ss {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kF64Waves = 4;
constexpr int kF64Threads = 64 * kF64Waves;
constexpr int kF64BandX = 128;   // 16 tiles of 8 columns
constexpr int kF64Rows = 16;     // 4 tile rows of 4

template <int RAD>
struct F64Geom {
    static constexpr int R1 = 8, R2 = 4, MB = 2;
    static constexpr int SROWS = kF64Rows + 2 * RAD;
    static constexpr int PITCH = kF64BandX + 2 * RAD + 1;  // doubles per slab row (odd: spreads banks)
};

__device__ inline int wrap64(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

template <int RAD, int KC>
__global__ __launch_bounds__(kF64Threads) void k_mma2d_f64(MmaArgs p) {
    using G = F64Geom<RAD>;
    __shared__ double slab[G::SROWS * G::PITCH];
    // block -> job, band, row block
    const int b = blockIdx.x;
    int j = 0;
    for (int t = 1; t < p.njobs; ++t) j += b >= p.job[t].item0 ? 1 : 0;
    const MmaJob &g = p.job[j];
    const int nbands = (g.nx + kF64BandX - 1) / kF64BandX;
    const int local = b - g.item0;
    const int X0 = (local % nbands) * kF64BandX, Y0 = (local / nbands) * kF64Rows;
    const double *in = static_cast<const double *>(g.in);
    double *out = static_cast<double *>(g.out);
    // slab: rows Y0-RAD.., columns X0-RAD.. (zero or wrapped outside)
    for (int e = threadIdx.x; e < G::SROWS * (kF64BandX + 2 * RAD); e += kF64Threads) {
        const int r = e / (kF64BandX + 2 * RAD), c = e % (kF64BandX + 2 * RAD);
        int gy = Y0 - RAD + r, gx = X0 - RAD + c;
        double v = 0.0;
        if (p.periodic) {
            v = in[(size_t)wrap64(gy, g.ny) * g.nx + wrap64(gx, g.nx)];
        } else if (gy >= 0 && gy < g.ny && gx >= 0 && gx < g.nx) {
            v = in[(size_t)gy * g.nx + gx];
        }
        slab[r * G::PITCH + c] = v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, q = lane >> 4;
    const double *ad = reinterpret_cast<const double *>(p.a_hi);
    double a[G::MB][KC];
    int off[KC];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        off[kc] = p.boff[kc * 4 + q];
#pragma unroll
        for (int mb = 0; mb < G::MB; ++mb) a[mb][kc] = ad[(mb * KC + kc) * 64 + lane];
    }
    __syncthreads();
    // wave w: tile row w; lane n: tile n of the row
    const double *tb = slab + (wave * G::R2) * G::PITCH + n * G::R1;
    d4 acc[G::MB];
#pragma unroll
    for (int mb = 0; mb < G::MB; ++mb) acc[mb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        const double bv = tb[off[kc]];
#pragma unroll
        for (int mb = 0; mb < G::MB; ++mb)
            acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb][kc], bv, acc[mb], 0, 0, 0);
    }
    // accumulator row 4i + q of M-block mb is tile output mb*16 + 4i + q
#pragma unroll
    for (int mb = 0; mb < G::MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = mb * 16 + 4 * i + q;
            const int y = Y0 + wave * G::R2 + o / G::R1, x = X0 + n * G::R1 + o % G::R1;
            if (y < g.ny && x < g.nx) out[(size_t)y * g.nx + x] = acc[mb][i];
        }
}

template <int RAD, int KC>
hipError_t launch_f64(MmaArgs &a, hipStream_t s) {
    if (a.njobs < 1 || a.njobs > kMaxJobs) return hipErrorInvalidValue;
    int blocks = 0;
    for (int j = 0; j < a.njobs; ++j) {
        a.job[j].item0 = blocks;
        blocks += ((a.job[j].nx + kF64BandX - 1) / kF64BandX) * ((a.job[j].ny + kF64Rows - 1) / kF64Rows);
    }
    a.total_items = blocks;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_mma2d_f64<RAD, KC>), dim3(blocks), dim3(kF64Threads), 0, s, a);
    return hipGetLastError();
}

}  // namespace

// Radius 1 at (8,4): K = 10 * 6 = 60 = 15 chunks of 4.
MmaLaunch find_mma2d_f64(int rad, int kc) {
    if (rad == 1 && kc == 15) return &launch_f64<1, 15>;
    return nullptr;
}

int mma2d_f64_pitch(int rad) { return rad == 1 ? F64Geom<1>::PITCH : 0; }

}  // namespace ss
