// 2-D stencil sweep as a structured-sparse (or dense) matrix product on
// gfx950 matrix cores.
//
// One output tile of r2 x r1 points is y = A'' * b'' where A'' (m' x K) is the
// permuted staircase coefficient matrix and b'' the tile's halo'd input patch
// gathered in the same K order (paper Sections 3.1-3.3).  Sixteen tiles form
// the N dimension of one MMA.  The FP32 state is split into hi + lo parts as it
// is staged into LDS; three products hi*hi + hi*lo + lo*hi accumulate in FP32
// (the lo parts carry a scale sigma that is divided out at the end).
//
// Operand layouts (gfx950, measured against dense MFMA):
//  * v_smfmac_f32_16x16x64_{f16,bf16}: lane l holds B column l%16 and the 16
//    K values 16*(l/16) + e; the compressed A row l%16 holds 8 values whose
//    pairs (2g', 2g'+1) belong to the 4-group of B lane group
//    2*((l/16)%2) + g'/2, element group 2*((l/16)/2) + g'%2, with 2-bit
//    positions in bits [2e+1:2e] of the index word.
//  * v_mfma_f32_16x16x32_{f16,bf16}: lane l holds A row l%16 / B column l%16
//    with K = 8*(l/16) + e.
//  * accumulators: lane l holds column l%16, rows 4*(l/16) + i.
//
// Gather: every 32-bit B register holds two horizontally adjacent patch
// elements starting at an even column, so a single 8-byte LDS read returns the
// hi pair and the lo pair (slab layout per column pair: hi0 hi1 lo0 lo1).
#include <hip/hip_runtime.h>

#include "kargs.hpp"
#include "kgeom.hpp"

namespace ss {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h16 __attribute__((ext_vector_type(16)));
typedef __bf16 bh8 __attribute__((ext_vector_type(8)));
typedef __bf16 bh16 __attribute__((ext_vector_type(16)));
typedef unsigned u8v __attribute__((ext_vector_type(8)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

template <int PART>
__device__ inline void split_pair(float x0, float x1, float sigma, unsigned *hi, unsigned *lo) {
    if constexpr (PART == kPartF16) {
        _Float16 h0 = (_Float16)x0, h1 = (_Float16)x1;
        _Float16 l0 = (_Float16)((x0 - (float)h0) * sigma);
        _Float16 l1 = (_Float16)((x1 - (float)h1) * sigma);
        *hi = (unsigned)__builtin_bit_cast(unsigned short, h0) |
              ((unsigned)__builtin_bit_cast(unsigned short, h1) << 16);
        *lo = (unsigned)__builtin_bit_cast(unsigned short, l0) |
              ((unsigned)__builtin_bit_cast(unsigned short, l1) << 16);
    } else {
        __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1;
        __bf16 l0 = (__bf16)((x0 - (float)h0) * sigma);
        __bf16 l1 = (__bf16)((x1 - (float)h1) * sigma);
        *hi = (unsigned)__builtin_bit_cast(unsigned short, h0) |
              ((unsigned)__builtin_bit_cast(unsigned short, h1) << 16);
        *lo = (unsigned)__builtin_bit_cast(unsigned short, l0) |
              ((unsigned)__builtin_bit_cast(unsigned short, l1) << 16);
    }
}

template <int MODE, int PART>
__device__ inline f4 mma(uint4 a, const unsigned *b, f4 c, unsigned idx) {
    if constexpr (MODE == kSparse) {
        u8v bv = {b[0], b[1], b[2], b[3], b[4], b[5], b[6], b[7]};
        u4v av = {a.x, a.y, a.z, a.w};
        if constexpr (PART == kPartF16)
            return __builtin_amdgcn_smfmac_f32_16x16x64_f16(__builtin_bit_cast(h8, av),
                                                           __builtin_bit_cast(h16, bv), c, (int)idx, 0, 0);
        else
            return __builtin_amdgcn_smfmac_f32_16x16x64_bf16(__builtin_bit_cast(bh8, av),
                                                            __builtin_bit_cast(bh16, bv), c, (int)idx, 0, 0);
    } else {
        u4v bv = {b[0], b[1], b[2], b[3]};
        u4v av = {a.x, a.y, a.z, a.w};
        if constexpr (PART == kPartF16)
            return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, av),
                                                         __builtin_bit_cast(h8, bv), c, 0, 0, 0);
        else
            return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bh8, av),
                                                          __builtin_bit_cast(bh8, bv), c, 0, 0, 0);
    }
}

__device__ inline int wrap_idx(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

template <int R1, int R2, int KC, int RAD, int MODE, int PART>
__global__ __launch_bounds__(kThreads) void k_mma2d(MmaArgs p) {
    using G = MmaGeom<R1, R2, RAD>;
    constexpr int MB = G::MB;
    constexpr int VPK = (MODE == kSparse) ? 8 : 4;  // B registers per K chunk
    __shared__ uint2 slab[G::SLAB_U16 / 4];
    unsigned short *lds = reinterpret_cast<unsigned short *>(slab);

    const float sigma = 1.0f / p.inv_sigma;
    const int X0 = blockIdx.x * kBandX;
    const int Y0 = blockIdx.y * G::WGH;

    // ---- stage the halo'd input slab, split into hi/lo parts
    for (int e = threadIdx.x; e < G::SROWS * G::CPS; e += kThreads) {
        const int row = e / G::CPS;
        const int cp = e - row * G::CPS;
        int gy = Y0 - RAD + row;
        int gx = X0 - RAD + 2 * cp;
        float v0 = 0.0f, v1 = 0.0f;
        if (p.periodic) {
            gy = wrap_idx(gy, p.ny);
            const int gx0 = wrap_idx(gx, p.nx), gx1 = wrap_idx(gx + 1, p.nx);
            const float *rowp = p.in + (size_t)gy * p.nx;
            v0 = rowp[gx0];
            v1 = rowp[gx1];
        } else if (gy >= 0 && gy < p.ny) {
            const float *rowp = p.in + (size_t)gy * p.nx;
            if (gx >= 0 && gx < p.nx) v0 = rowp[gx];
            if (gx + 1 >= 0 && gx + 1 < p.nx) v1 = rowp[gx + 1];
        }
        unsigned hi, lo;
        split_pair<PART>(v0, v1, sigma, &hi, &lo);
        const int slot = pair_slot(cp, G::F, G::S);
        slab[(row * G::PITCH + 4 * slot) / 4] = make_uint2(hi, lo);
    }

    // ---- per-lane constants: gather offsets and A fragments
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = lane & 15;
    const int q = lane >> 4;
    const int tx_t = n % G::NBX;
    const int ty_t = n / G::NBX;

    int off[KC][VPK];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int v = 0; v < VPK; ++v) off[kc][v] = p.boff[(kc * 4 + q) * VPK + v];

    uint4 ahi[MB][KC], alo[MB][KC];
    unsigned aidx[MB][KC];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const int t = (mb * KC + kc) * 64 + lane;
            ahi[mb][kc] = p.a_hi[t];
            alo[mb][kc] = p.a_lo[t];
            aidx[mb][kc] = (MODE == kSparse) ? p.a_idx[t] : 0u;
        }

    __syncthreads();

#pragma unroll 1
    for (int nbi = 0; nbi < kNbw; ++nbi) {
        const int nb = wave * kNbw + nbi;
        const int srow0 = nb * G::NBH + ty_t * R2;
        const int base = srow0 * G::PITCH + 4 * tx_t;
        f4 accm[MB], accc[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            accm[mb] = f4{0.f, 0.f, 0.f, 0.f};
            accc[mb] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            unsigned bh[VPK], bl[VPK];
#pragma unroll
            for (int v = 0; v < VPK; ++v) {
                const uint2 t = slab[(base + off[kc][v]) >> 2];
                bh[v] = t.x;
                bl[v] = t.y;
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                accm[mb] = mma<MODE, PART>(ahi[mb][kc], bh, accm[mb], aidx[mb][kc]);
                accc[mb] = mma<MODE, PART>(ahi[mb][kc], bl, accc[mb], aidx[mb][kc]);
                accc[mb] = mma<MODE, PART>(alo[mb][kc], bh, accc[mb], aidx[mb][kc]);
            }
        }
        // ---- write back: accumulator rows 4q..4q+3 of M-block mb are outputs
        // mb*16 + 4q + i of the tile, four consecutive x positions.
        const int ybase = Y0 + nb * G::NBH + ty_t * R2;
        const int xbase = X0 + tx_t * R1;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int o = mb * 16 + 4 * q;
            const int gy = ybase + o / R1;
            const int gx = xbase + o % R1;
            if (gy >= p.ny) continue;
            f4 y;
#pragma unroll
            for (int i = 0; i < 4; ++i) y[i] = accm[mb][i] + accc[mb][i] * p.inv_sigma;
            float *dst = p.out + (size_t)gy * p.nx + gx;
            if ((p.nx & 3) == 0 && gx + 3 < p.nx) {
                *reinterpret_cast<f4 *>(dst) = y;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (gx + i < p.nx) dst[i] = y[i];
            }
        }
    }
}

template <int R1, int R2, int KC, int RAD, int MODE, int PART>
static hipError_t launch_mma2d(const MmaArgs &a, hipStream_t s) {
    using G = MmaGeom<R1, R2, RAD>;
    dim3 grid((a.nx + kBandX - 1) / kBandX, (a.ny + G::WGH - 1) / G::WGH);
    hipLaunchKernelGGL((k_mma2d<R1, R2, KC, RAD, MODE, PART>), grid, dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

struct MmaEntry {
    MmaKey key;
    MmaLaunch fn;
    int wgh, pitch, F, S;
};

#define SS_MMA(R1, R2, KC, RAD, MODE, PART)                                                         \
    {{R1, R2, KC, RAD, MODE, PART},                                                                 \
     &launch_mma2d<R1, R2, KC, RAD, MODE, PART>,                                                    \
     MmaGeom<R1, R2, RAD>::WGH, MmaGeom<R1, R2, RAD>::PITCH, MmaGeom<R1, R2, RAD>::F,               \
     MmaGeom<R1, R2, RAD>::S}

// Instantiated layouts: k = 3 (radius 1) at (8,8) and (16,4): sparse K 128
// (2 chunks of 64), dense K 128 (4 chunks of 32), binary16 and bfloat16 parts.
static const MmaEntry kMmaTable[] = {
    SS_MMA(8, 8, 2, 1, kSparse, kPartF16),  SS_MMA(8, 8, 4, 1, kDense, kPartF16),
    SS_MMA(16, 4, 2, 1, kSparse, kPartF16), SS_MMA(16, 4, 4, 1, kDense, kPartF16),
    SS_MMA(8, 8, 2, 1, kSparse, kPartBF16), SS_MMA(8, 8, 4, 1, kDense, kPartBF16),
    SS_MMA(16, 4, 2, 1, kSparse, kPartBF16), SS_MMA(16, 4, 4, 1, kDense, kPartBF16),
};

MmaLaunch find_mma2d(const MmaKey &k) {
    for (const auto &e : kMmaTable)
        if (e.key.r1 == k.r1 && e.key.r2 == k.r2 && e.key.kc == k.kc && e.key.rad == k.rad &&
            e.key.mode == k.mode && e.key.part == k.part)
            return e.fn;
    return nullptr;
}

bool mma2d_geometry(const MmaKey &k, int *wgh, int *pitch, int *F, int *S) {
    for (const auto &e : kMmaTable)
        if (e.key.r1 == k.r1 && e.key.r2 == k.r2 && e.key.kc == k.kc && e.key.rad == k.rad &&
            e.key.mode == k.mode && e.key.part == k.part) {
            *wgh = e.wgh;
            *pitch = e.pitch;
            *F = e.F;
            *S = e.S;
            return true;
        }
    return false;
}

}  // namespace ss
