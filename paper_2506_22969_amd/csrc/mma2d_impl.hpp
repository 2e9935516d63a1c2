// Building blocks of the 2-D slab pipelines on gfx950 (shared by the
// matrix kernels of mma2d_conv.hpp, the direct LDS kernels of direct2d.hip,
// and the 1-D and 3-D kernels): binary16 / bfloat16 splitting, the MMA
// wrappers, buffer descriptors, boundary index wrapping, explicit vmcnt
// waits, LDS DMA, and the slab loads of the 2-D direct kernels (FP32 rows
// with a halo staging strip, or bfloat16 planes rows whose hi and lo dword
// pairs alternate).
#pragma once

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
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));

// Split two FP32 values into packed hi parts and sigma-scaled lo parts,
// rounding to nearest even.  x - hi is exact in FP32.  binary16: one packed
// conversion for the hi pair, x - hi by mixed-precision FMAs that read the
// binary16 halves directly, and (x - hi) * sigma rounded into the lo and hi
// halves of the lo word.  bfloat16: packed conversions both ways.
template <int PART>
__device__ inline void split2(float x0, float x1, float sigma, unsigned *hi, unsigned *lo) {
    const f2v x = {x0, x1};
    if constexpr (PART == kPartF16) {
        const unsigned h = __builtin_bit_cast(unsigned, __builtin_convertvector(x, h2v));
        float d0, d1;
        asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(d0) : "v"(h), "v"(x0));
        asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(d1) : "v"(h), "v"(x1));
        unsigned l;
        asm("v_fma_mixlo_f16 %0, %1, %2, 0" : "=v"(l) : "v"(d0), "v"(sigma));
        asm("v_fma_mixhi_f16 %0, %1, %2, 0" : "+v"(l) : "v"(d1), "v"(sigma));
        *hi = h;
        *lo = l;
    } else {
        const b2v h = __builtin_convertvector(x, b2v);
        const f2v r = (x - __builtin_convertvector(h, f2v)) * sigma;
        *hi = __builtin_bit_cast(unsigned, h);
        *lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, b2v));
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

// Raw buffer descriptor word 3 for gfx9-family (gfx950) and an offset past
// any descriptor's range (out-of-range buffer stores are dropped).
constexpr int kRsrcWord3 = 0x00020000;
constexpr unsigned kOob = 0x80000000u;

// Buffer descriptor over `bytes` bytes at `base` (wave-uniform values, read
// from lane 0 so that the descriptor is known to live in scalar registers).
__device__ inline __amdgpu_buffer_rsrc_t uniform_rsrc(void *base, int bytes) {
    const unsigned long long b = (unsigned long long)base;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    void *ub = (void *)(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(ub, 0, __builtin_amdgcn_readfirstlane(bytes), kRsrcWord3);
}

// Boundary handling compiled into a kernel: zero halo; periodic with at most
// one wrap per index (grid at least as large as a slab); periodic general.
enum Bc { kBcZero = 0, kBcWrap1 = 1, kBcWrapN = 2 };

template <int BC>
__device__ inline int wrap(int i, int n) {
    if constexpr (BC == kBcWrap1) {
        i += i < 0 ? n : 0;
        i -= i >= n ? n : 0;
    } else if constexpr (BC == kBcWrapN) {
        i %= n;
        i += i < 0 ? n : 0;
    }
    return i;
}

// s_waitcnt with only vmcnt constrained (gfx9 encoding: vmcnt[3:0] in bits
// 3:0 and vmcnt[5:4] in bits 15:14; expcnt and lgkmcnt left at their maxima).
// vmcnt counts a wave's VMEM operations in issue order and a wave cannot have
// more than 63 outstanding (issue waits), so waiting for "at most 63 newer
// operations" also covers an operation followed by more than 63.
template <int N>
__device__ inline void wait_vmcnt() {
    static_assert(N >= 0, "vmcnt range");
    constexpr int C = N < 63 ? N : 63;
    __builtin_amdgcn_s_waitcnt((C & 15) | ((C >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Slab loads of one work item of the 2-D direct kernels (item geometry of
// an (8,8) MmaGeom): DRW slab rows per wave, DMA_PER_ROW transfers per row,
// D VMEM loads per wave per item.
template <int R1, int R2, int RAD, int STATE, bool VEC>
struct Pipe {
    using G = MmaGeom<R1, R2, RAD, STATE>;
    static constexpr int DRW = (G::SROWS + kWaves - 1) / kWaves;      // slab rows each wave loads
    // LDS-DMA operations per slab row: FP32 one 16-byte transfer per lane
    // (or four 4-byte ones when rows are not 16-byte aligned); planes four
    // 4-byte transfers per lane and one by 16 lanes (272 dwords)
    static constexpr int DMA_PER_ROW = STATE == kStatePlanes ? 5 : (VEC ? 1 : kBandX / 64);
    static constexpr int D = DRW * DMA_PER_ROW + G::HOPS;               // VMEM loads per wave per item
};

// LDS DMA: each active lane copies 16 (or 4) bytes from its global address to
// LDS at lds_addr + 16*lane (or 4*lane), lane being the lane id in the wave.
// Written as inline assembly so that the compiler does not track these
// transfers: the pipeline waits for them explicitly with s_waitcnt vmcnt
// before the barrier that publishes a slab.
// The LDS address is wave-uniform; readfirstlane keeps it in an SGPR even
// where the compiler computed it with vector instructions.
__device__ inline void lds_dma16(const void *src, unsigned lds_addr) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(src), "s"(__builtin_amdgcn_readfirstlane(lds_addr))
                 : "memory", "m0");
}
__device__ inline void lds_dma4(const void *src, unsigned lds_addr) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %0, off"
                 :
                 : "v"(src), "s"(__builtin_amdgcn_readfirstlane(lds_addr))
                 : "memory", "m0");
}
// The same transfers from a wave-uniform base plus a 32-bit per-lane byte
// offset (the scalar-base form of the instruction).
__device__ inline void lds_dma16_at(const void *sbase, unsigned off, unsigned lds_addr) {
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
                 :
                 : "v"(off), "s"(sbase), "s"(__builtin_amdgcn_readfirstlane(lds_addr))
                 : "memory", "m0");
}
__device__ inline void lds_dma4_at(const void *sbase, unsigned off, unsigned lds_addr) {
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dword %0, %1"
                 :
                 : "v"(off), "s"(sbase), "s"(__builtin_amdgcn_readfirstlane(lds_addr))
                 : "memory", "m0");
}
__device__ inline unsigned lds_addr_of(const void *p) {
    return (unsigned)(size_t)(const __attribute__((address_space(3))) char *)p;
}

// Issue the loads of one work item.  FP32: the 256 interior columns of every
// slab row (one 64-lane 16-byte transfer per row, or four 64-lane 4-byte
// transfers when rows are not 16-byte aligned); halo columns go to a staging
// strip by 4-byte transfers (put_halo moves them into place).  Planes: each
// slab row, halo included, by 4-byte transfers whose lanes alternate between
// the hi and the lo plane.  Rows or columns outside a zero-halo grid read
// from a zero page.  Every wave issues
// the same number of transfers for every item (item and row indices are
// clamped), which is what the explicit waits count on.
template <int R1, int R2, int RAD, int STATE, bool VEC, int BC>
__device__ inline void issue_item(const void *zero_block, const MmaJob &g, char *slab, unsigned *strip, int X0,
                                  int Y0) {
    using G = MmaGeom<R1, R2, RAD, STATE>;
    using P = Pipe<R1, R2, RAD, STATE, VEC>;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    X0 = __builtin_amdgcn_readfirstlane(X0);
    Y0 = __builtin_amdgcn_readfirstlane(Y0);
    const char *zeros = static_cast<const char *>(zero_block);
#pragma unroll
    for (int d = 0; d < P::DRW; ++d) {
        const int r = min(wave + d * kWaves, G::SROWS - 1);
        const int gy = wrap<BC>(Y0 - RAD + r, g.ny);
        const bool row_ok = BC != kBcZero || (gy >= 0 && gy < g.ny);
        if constexpr (STATE == kStatePlanes) {
            // dword 64h + lane of the row: plane lane & 1, values
            // X0 - HLB + 64h + (lane & ~1) and the next (rows are a multiple
            // of 8 values, so a pair is all in or all out of the grid)
            const unsigned short *in = static_cast<const unsigned short *>(g.in);
            const size_t plane = (size_t)g.ny * g.nx;
            const unsigned dst = lds_addr_of(slab + r * G::RBD * 4);
#pragma unroll
            for (int h = 0; h < 5; ++h) {
                if (h < 4 || lane < 16) {
                    const int gx = wrap<BC>(X0 - G::HLB + 64 * h + (lane & ~1), g.nx);
                    const bool ok = BC != kBcZero || (row_ok && gx >= 0 && gx < g.nx);
                    const void *src = ok ? (const void *)(in + (lane & 1) * plane + (size_t)gy * g.nx + gx)
                                         : (const void *)(zeros + 4 * lane);
                    lds_dma4(src, dst + 256 * h);
                }
            }
        } else {
            const float *in = static_cast<const float *>(g.in);
            const float *zf = reinterpret_cast<const float *>(zeros);
            const unsigned dst = lds_addr_of(reinterpret_cast<float *>(slab) + r * G::CPITCH + G::HL);
            if constexpr (VEC) {
                const int gx = wrap<BC>(X0 + 4 * lane, g.nx);
                const bool ok = BC != kBcZero || (row_ok && gx < g.nx);
                const float *src = ok ? in + (size_t)gy * g.nx + gx : zf + 4 * lane;
                lds_dma16(src, dst);
            } else {
#pragma unroll
                for (int h = 0; h < P::DMA_PER_ROW; ++h) {
                    const int gx = wrap<BC>(X0 + 64 * h + lane, g.nx);
                    const bool ok = BC != kBcZero || (row_ok && gx < g.nx);
                    const float *src = ok ? in + (size_t)gy * g.nx + gx : zf + lane;
                    lds_dma4(src, dst + 256 * h);
                }
            }
        }
    }
    if constexpr (G::NHALO > 0) {
#pragma unroll
    for (int h = 0; h < G::HOPS; ++h) {
        const int base = (h * kWaves + wave) * 64;
        const int e = min(base + lane, G::NHALO - 1);
        const int r = e / G::HALO_ROW, j = e % G::HALO_ROW;
        const int gy = wrap<BC>(Y0 - RAD + r, g.ny);
        const int gx = wrap<BC>(j < RAD ? X0 - RAD + j : X0 + kBandX + (j - RAD), g.nx);
        const bool ok = BC != kBcZero || (gy >= 0 && gy < g.ny && gx >= 0 && gx < g.nx);
        const float *in = static_cast<const float *>(g.in);
        const void *src = ok ? (const void *)(in + (size_t)gy * g.nx + gx) : (const void *)(zeros + 4 * lane);
        lds_dma4(src, lds_addr_of(strip + base));
    }
    }
}

// Move an item's halo columns from the staging strip into the slab.
template <int R1, int R2, int RAD, int STATE>
__device__ inline void put_halo(char *slab, const unsigned *strip) {
    using G = MmaGeom<R1, R2, RAD, STATE>;
    static_assert(G::NHALO > 0, "FP32 slabs only");
    for (int e = threadIdx.x; e < G::NHALO; e += kThreads) {
        const int r = e / G::HALO_ROW, j = e % G::HALO_ROW;
        const int c = j < RAD ? G::HL - RAD + j : G::HL + kBandX + (j - RAD);
        reinterpret_cast<unsigned *>(slab)[r * G::CPITCH + c] = strip[e];
    }
}

// Compute units and XCDs of the current device (queried once per device).
hipError_t device_shape(int *cus, int *xcds);

}  // namespace ss

namespace ss {

// An instantiated kernel: its key, launch, rows per work item, gather row
// pitch, and for the converted slabs (pw > 0) the dwords per pair and the
// pairs between row gaps.
struct MmaEntry {
    MmaKey key;
    MmaLaunch fn;
    int wgh, row;
    int pw, padg;
};

// Tables of the instantiating translation units.
const MmaEntry *mma_table_f32_r1(int *n);
const MmaEntry *mma_table_f32_r2(int *n);
const MmaEntry *mma_table_f32_r3(int *n);
const MmaEntry *mma_table_f16(int *n);
const MmaEntry *mma_table_planes(int *n);
const MmaEntry *mma_table_planes3(int *n);

// Points of a grid that the band of a fused zero-halo launch covers (none
// when b = 0): rows within b of the top or bottom edge, columns [0, bl) and
// [br, nx) -- the band's b columns widened to whole groups of four, the
// granularity of the products' stores.
struct BandBounds {
    int b, bl, br;
};

__device__ inline BandBounds band_bounds(const MmaArgs &p, const MmaJob &g) {
    if (p.edge_steps < 2) return BandBounds{0, 0, g.nx};
    const int b = p.edge_rad * (p.edge_steps - 1);
    return BandBounds{b, (b + 3) & ~3, max(0, (g.nx - b) & ~3)};
}

}  // namespace ss
