// 2-D stencil sweep as a structured-sparse (or dense) matrix product on
// gfx950 matrix cores (kernel template; instantiated by mma2d_*.hip).
//
// One output tile of r2 x r1 points is y = A'' * b'' where A'' (m' x K) is the
// permuted staircase coefficient matrix and b'' the tile's halo'd input patch
// gathered in the same K order (paper Sections 3.1-3.3).  Sixteen tiles form
// the N dimension of one MMA.  The state is staged into LDS as stored (FP32,
// or bfloat16 hi and lo planes) and turned into hi + lo B operands as it is
// gathered into registers; three products hi*hi + hi*lo + lo*hi accumulate in
// FP32 (the lo parts carry a scale sigma that is divided out at the end).
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
// elements (the 4-group layout [P0.a, P1.a, P0.b, P1.b] puts the column-t and
// column-(t+1) elements of a block pair side by side), so one two-dword LDS
// read feeds one hi and one lo register: two FP32 values split in registers,
// or, on the planes state whose slab rows interleave hi and lo dword pairs,
// the pair's hi and lo dwords (even radius: the pair starts at an even
// column), or two such reads and two byte aligns (odd radius).
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

// Per-workgroup pipeline geometry of the 2-D MMA kernel.
template <int R1, int R2, int RAD, int STATE, bool VEC>
struct Pipe {
    using G = MmaGeom<R1, R2, RAD, STATE>;
    static constexpr int DRW = (G::SROWS + kWaves - 1) / kWaves;      // slab rows each wave loads
    // LDS-DMA operations per slab row: FP32 one 16-byte transfer per lane
    // (or four 4-byte ones when rows are not 16-byte aligned); planes four
    // 4-byte transfers per lane and one by 16 lanes (272 dwords)
    static constexpr int DMA_PER_ROW = STATE == kStatePlanes ? 5 : (VEC ? 1 : kBandX / 64);
    static constexpr int D = DRW * DMA_PER_ROW + G::HOPS;               // VMEM loads per wave per item
    static constexpr int STORES_PER_MB = STATE == kStatePlanes ? 2 : (VEC ? 1 : 4);
    static constexpr int M = G::U * G::MB * STORES_PER_MB;              // VMEM stores per wave per item
    // VMEM operations issued after item s's last load when it is consumed:
    // the loads of the NSLAB-2 items issued after it and the stores of the
    // min(s, NSLAB-1) items computed since
    template <int S>
    static constexpr int W = (G::NSLAB - 2) * D + (S < G::NSLAB - 1 ? S : G::NSLAB - 1) * M;
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

// Gather offset (bytes) of B register v of a K chunk: two 16-bit offsets
// per word.  The word passes through an empty asm that takes a loop-varying
// value (the item and unit number), so that the unpacked offsets are not hoisted out of
// the loop and kept live (which would undo the packing); the asm touches no
// memory, so the LDS reads around it can still be scheduled freely.
template <int VPK>
__device__ inline int gather_off(const unsigned (&o2)[VPK / 2], int v, int salt) {
    unsigned w = o2[v >> 1];
    asm("" : "+v"(w) : "s"(salt));
    return (v & 1) ? (int)(w >> 16) : (int)(w & 0xffffu);
}

// Multiply one work item out of its LDS slab and write its outputs.  Wave w
// owns units (w / NCOLS) * U + u of unit column w % NCOLS: 16 tiles of
// R2 x R1 outputs each.
template <int R1, int R2, int KC, int RAD, int MODE, int PART, int STATE, bool VEC>
__device__ inline void compute_item(float inv_sigma, const MmaJob &g, const char *slab,
                                    const uint4 (&ahi)[R1 * R2 / 16][KC], const uint4 (&alo)[R1 * R2 / 16][KC],
                                    const unsigned (&aidx)[R1 * R2 / 16][KC],
                                    const unsigned (&off2)[KC][(MODE == kSparse) ? 4 : 2], int X0, int Y0,
                                    float sigma, int salt) {
    using G = MmaGeom<R1, R2, RAD, STATE>;
    constexpr int MB = G::MB;
    constexpr int VPK = (MODE == kSparse) ? 8 : 4;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nb = wave / G::NCOLS;           // unit row group of the item
    const int nbc = wave % G::NCOLS;          // unit column of the band
    const int n = lane & 15;
    const int q = lane >> 4;
    const int tx_t = n % G::NBX;
    const int ty_t = n / G::NBX;
    // X0, Y0 are uniform; saying so keeps the store descriptors in SGPRs
    X0 = __builtin_amdgcn_readfirstlane(X0);
    Y0 = __builtin_amdgcn_readfirstlane(Y0);
    const int rows_left = min(G::WGH, g.ny - Y0);
    const int xbase = X0 + nbc * G::UW + tx_t * R1;
#pragma unroll 1
    for (int u = 0; u < G::U; ++u) {
        const int urow = (nb * G::U + u) * G::NBH;   // first row of the unit in the item
        const int srow0 = urow + ty_t * R2;          // tile's first row (slab rows start RAD above)
        // hi*hi, hi*lo and lo*hi accumulate separately (no back-to-back
        // dependent MMAs)
        f4 accm[MB], acc1[MB], acc2[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            accm[mb] = f4{0.f, 0.f, 0.f, 0.f};
            acc1[mb] = f4{0.f, 0.f, 0.f, 0.f};
            acc2[mb] = f4{0.f, 0.f, 0.f, 0.f};
        }
        // byte address in the slab of the tile's patch origin (planes: of the
        // dword pair holding its first column); gather offsets are in bytes
        // from it
        const int c0 = G::MARGIN - RAD + nbc * G::UW + tx_t * R1;
        const int tbo = STATE == kStatePlanes ? srow0 * G::ROW + (c0 >> 1) * 8 : (srow0 * G::ROW + c0) * 4;
        const char *tb = slab + tbo;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            unsigned bh[VPK], bl[VPK];
            if constexpr (STATE == kStatePlanes) {
#pragma unroll
                for (int v = 0; v < VPK; ++v) {
                    if constexpr (G::PAIR_DWORD) {
                        // hi and lo dwords of the pair, side by side
                        const unsigned *w = reinterpret_cast<const unsigned *>(tb + gather_off<VPK>(off2[kc], v, salt + u));
                        bh[v] = w[0];
                        bl[v] = w[1];
                    } else {
                        // the pair may start at an odd value (offset bit 1):
                        // two dword pairs and a byte align (offset arithmetic
                        // stays relative to the slab, so the reads remain LDS
                        // reads)
                        const int ai = tbo + gather_off<VPK>(off2[kc], v, salt + u);
                        const unsigned *w = reinterpret_cast<const unsigned *>(slab + (ai & ~3));
                        const unsigned sh = (unsigned)(ai & 2);
                        bh[v] = __builtin_amdgcn_alignbyte(w[2], w[0], sh);
                        bl[v] = __builtin_amdgcn_alignbyte(w[3], w[1], sh);
                    }
                }
            } else {
#pragma unroll
                for (int v = 0; v < VPK; ++v) {
                    const float *src = reinterpret_cast<const float *>(tb + gather_off<VPK>(off2[kc], v, salt + u));
                    split2<PART>(src[0], src[1], sigma, &bh[v], &bl[v]);
                }
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) accm[mb] = mma<MODE, PART>(ahi[mb][kc], bh, accm[mb], aidx[mb][kc]);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc1[mb] = mma<MODE, PART>(ahi[mb][kc], bl, acc1[mb], aidx[mb][kc]);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc2[mb] = mma<MODE, PART>(alo[mb][kc], bh, acc2[mb], aidx[mb][kc]);
        }
        // write back: accumulator rows 4q..4q+3 of M-block mb are outputs
        // mb*16 + 4q + i of the tile, four consecutive x positions.  Buffer
        // stores with an out-of-range offset drop the write, so every store
        // is issued.
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int o = mb * 16 + 4 * q;
            const int gyr = srow0 + o / R1;
            const int gx = xbase + o % R1;
            float ys[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) ys[i] = accm[mb][i] + (acc1[mb][i] + acc2[mb][i]) * inv_sigma;
            const bool row_ok = gyr < rows_left;
            if constexpr (STATE == kStatePlanes) {
                // bfloat16 hi = RNE(y), lo = RNE(y - hi); rows are a
                // multiple of 8 values, so the four outputs are all in or all out
                unsigned short h[4], l[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const __bf16 hb = (__bf16)ys[i];
                    const __bf16 lb = (__bf16)(ys[i] - (float)hb);
                    h[i] = __builtin_bit_cast(unsigned short, hb);
                    l[i] = __builtin_bit_cast(unsigned short, lb);
                }
                const u2v hv = {(unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16)};
                const u2v lv = {(unsigned)l[0] | ((unsigned)l[1] << 16), (unsigned)l[2] | ((unsigned)l[3] << 16)};
                unsigned short *out = static_cast<unsigned short *>(g.out);
                const size_t plane = (size_t)g.ny * g.nx;
                const __amdgpu_buffer_rsrc_t rh = uniform_rsrc(out + (size_t)Y0 * g.nx, rows_left * g.nx * 2);
                const __amdgpu_buffer_rsrc_t rl =
                    uniform_rsrc(out + plane + (size_t)Y0 * g.nx, rows_left * g.nx * 2);
                const unsigned o2 = row_ok && gx < g.nx ? (unsigned)(gyr * g.nx + gx) * 2u : kOob;
                __builtin_amdgcn_raw_buffer_store_b64(hv, rh, o2, 0, 0);
                __builtin_amdgcn_raw_buffer_store_b64(lv, rl, o2, 0, 0);
            } else {
                float *out = static_cast<float *>(g.out);
                const __amdgpu_buffer_rsrc_t orsrc = uniform_rsrc(out + (size_t)Y0 * g.nx, rows_left * g.nx * 4);
                if constexpr (VEC) {
                    const u4v yv = {__float_as_uint(ys[0]), __float_as_uint(ys[1]), __float_as_uint(ys[2]),
                                    __float_as_uint(ys[3])};
                    const unsigned o4 = row_ok && gx < g.nx ? (unsigned)(gyr * g.nx + gx) * 4u : kOob;
                    __builtin_amdgcn_raw_buffer_store_b128(yv, orsrc, o4, 0, 0);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const unsigned o1 =
                            row_ok && gx + i < g.nx ? (unsigned)(gyr * g.nx + gx + i) * 4u : kOob;
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(ys[i]), orsrc, o1, 0, 0);
                    }
                }
            }
        }
    }
}

// Persistent sweep kernel, one workgroup per CU.  Work items are (256-column
// band, 32-row block) pairs in row-block-major order.  Workgroups are dealt
// to the XCDs round robin (workgroup g runs on XCD g mod X); each XCD takes
// one contiguous range of items, in proportion to its workgroup count, and
// its workgroups interleave over that range, so that the rows an item shares
// with its neighbours are fetched into the same L2 at about the same time.
// NSLAB LDS slabs rotate: while item s is multiplied out of one, the inputs
// of the next NSLAB-1 items stream into the others by LDS DMA, which keeps
// about 100 KB per CU in flight without holding it in registers.
template <int R1, int R2, int KC, int RAD, int MODE, int PART, int STATE, bool VEC, int BC>
__global__ __launch_bounds__(kThreads, 1) void k_mma2d(MmaArgs p) {
    using G = MmaGeom<R1, R2, RAD, STATE>;
    using P = Pipe<R1, R2, RAD, STATE, VEC>;
    constexpr int MB = G::MB;
    constexpr int VPK = (MODE == kSparse) ? 8 : 4;  // B registers per K chunk
    constexpr int NS = G::NSLAB;
    __shared__ __attribute__((aligned(16))) char lds[NS * (G::SLAB_BYTES + 4 * G::HSTRIP)];
    auto slab = [&](int i) { return lds + i * G::SLAB_BYTES; };
    auto strip = [&](int i) { return reinterpret_cast<unsigned *>(lds + NS * G::SLAB_BYTES) + i * G::HSTRIP; };

    const float sigma = 1.0f / p.inv_sigma;
    const float inv_sigma = p.inv_sigma;
    const void *zero_block = p.zeros;
    const int nxcd = p.nxcd;
    const int nwg = gridDim.x;
    const int xcd = blockIdx.x % nxcd;
    const int stride = nwg / nxcd + (xcd < nwg % nxcd ? 1 : 0);       // workgroups on this XCD
    const int before = xcd * (nwg / nxcd) + min(xcd, nwg % nxcd);     // ... on the XCDs before it
    const int range_begin = (int)((long long)p.total_items * before / nwg);
    const int total = (int)((long long)p.total_items * (before + stride) / nwg);  // end of the range
    const int first = range_begin + blockIdx.x / nxcd;
    if (first >= total) return;

    const int lane = threadIdx.x & 63;
    const int q = lane >> 4;
    // gather offsets (below 2^16 bytes for every instantiated geometry)
    unsigned off2[KC][VPK / 2];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int v = 0; v < VPK; v += 2)
            off2[kc][v / 2] = (unsigned)p.boff[(kc * 4 + q) * VPK + v] |
                              ((unsigned)p.boff[(kc * 4 + q) * VPK + v + 1] << 16);
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
    // the table loads above are the only VMEM loads the compiler tracks
    wait_vmcnt<0>();

    // item of pipeline step s (clamped: loads past the end of the range
    // re-read its last item and are never consumed), its job and the item's
    // origin in the job
    auto item = [&](int s) { return min(first + s * stride, total - 1); };
    auto locate = [&](int it, int &j, int &X0, int &Y0) {
        j = 0;
        for (int t = 1; t < p.njobs; ++t) j += it >= p.job[t].item0 ? 1 : 0;
        const int nbands = (p.job[j].nx + kBandX - 1) / kBandX;
        const int local = it - p.job[j].item0;
        X0 = (local % nbands) * kBandX;
        Y0 = (local / nbands) * G::WGH;
    };
    auto issue = [&](int s) {
        int j, X0, Y0;
        locate(item(s), j, X0, Y0);
        const int i = s % NS;
        // a copy in registers: the transfers' memory clobbers would
        // otherwise make every use reload the job from the argument block
        const MmaJob g = p.job[j];
        issue_item<R1, R2, RAD, STATE, VEC, BC>(zero_block, g, slab(i), strip(i), X0, Y0);
    };
#pragma unroll
    for (int s = 0; s < NS - 1; ++s) issue(s);

#pragma unroll 1
    for (int s = 0;; ++s) {
        // wait for item s's transfers (every wave's, after the barrier),
        // move an FP32 halo into place, refill the slab item s-1 used with item
        // s+NS-1, multiply item s
        switch (s) {
            case 0: wait_vmcnt<P::template W<0>>(); break;
            case 1: wait_vmcnt<P::template W<1>>(); break;
            case 2: wait_vmcnt<P::template W<2>>(); break;
            default: wait_vmcnt<P::template W<3>>(); break;
        }
        const int cur = s % NS;
        __builtin_amdgcn_s_barrier();
        if constexpr (G::NHALO > 0) {
            put_halo<R1, R2, RAD, STATE>(slab(cur), strip(cur));
            __builtin_amdgcn_s_waitcnt(0xC07F);      // lgkmcnt(0): halo writes done
            __builtin_amdgcn_s_barrier();
        }
        issue(s + NS - 1);
        int j, X0, Y0;
        locate(item(s), j, X0, Y0);
        const MmaJob g = p.job[j];
        compute_item<R1, R2, KC, RAD, MODE, PART, STATE, VEC>(inv_sigma, g, slab(cur), ahi, alo, aidx, off2, X0,
                                                               Y0, sigma, s * G::U);
        if (first + (s + 1) * stride >= total) break;
    }
    // the pipeline always runs NS-1 items ahead: let those transfers land
    // before the workgroup's LDS is released
    wait_vmcnt<0>();
}

// Compute units and XCDs of the current device (queried once per device).
hipError_t device_shape(int *cus, int *xcds);

template <int R1, int R2, int KC, int RAD, int MODE, int PART, int STATE, bool VEC, int BC>
static hipError_t launch_bc(const MmaArgs &a, hipStream_t s) {
    int cus = 0, xcds = 0;
    if (const hipError_t e = device_shape(&cus, &xcds); e != hipSuccess) return e;
    MmaArgs b = a;
    b.nxcd = xcds;
    // one workgroup per CU, never more workgroups than items
    const int g = a.total_items < cus ? a.total_items : cus;
    hipLaunchKernelGGL((k_mma2d<R1, R2, KC, RAD, MODE, PART, STATE, VEC, BC>), dim3(g), dim3(kThreads), 0, s,
                       b);
    return hipGetLastError();
}

// Number the jobs' work items, then pick the kernel variant every job of the
// launch can use: 16-byte-aligned rows or not, and the cheapest boundary
// handling valid for all of them.  The planes state has only 16-byte-aligned
// variants (rows a multiple of 8 values; the planner checks).
template <int R1, int R2, int KC, int RAD, int MODE, int PART, int STATE>
static hipError_t launch_mma2d(MmaArgs &a, hipStream_t s) {
    using G = MmaGeom<R1, R2, RAD, STATE>;
    if (a.njobs < 1 || a.njobs > kMaxJobs) return hipErrorInvalidValue;
    int items = 0;
    bool vec = true, wrap1 = true;
    for (int j = 0; j < a.njobs; ++j) {
        const MmaJob &g = a.job[j];
        a.job[j].item0 = items;
        items += ((g.nx + kBandX - 1) / kBandX) * ((g.ny + G::WGH - 1) / G::WGH);
        vec = vec && (g.nx % (STATE == kStatePlanes ? 8 : 4)) == 0;
        // one wrap suffices when every index is within one grid length
        wrap1 = wrap1 && g.ny >= G::SROWS &&
                g.nx >= kBandX + (STATE == kStatePlanes ? 2 * G::HLB : 2 * RAD + 2);
    }
    a.total_items = items;
    if (items == 0) return hipSuccess;
    if constexpr (STATE == kStatePlanes) {
        if (!vec) return hipErrorInvalidValue;
        if (!a.periodic) return launch_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcZero>(a, s);
        if (wrap1) return launch_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcWrap1>(a, s);
        return launch_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcWrapN>(a, s);
    } else {
        if (vec) {
            if (!a.periodic) return launch_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcZero>(a, s);
            if (wrap1) return launch_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcWrap1>(a, s);
            return launch_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcWrapN>(a, s);
        }
        if (!a.periodic) return launch_bc<R1, R2, KC, RAD, MODE, PART, STATE, false, kBcZero>(a, s);
        if (wrap1) return launch_bc<R1, R2, KC, RAD, MODE, PART, STATE, false, kBcWrap1>(a, s);
        return launch_bc<R1, R2, KC, RAD, MODE, PART, STATE, false, kBcWrapN>(a, s);
    }
}

#define SS_MMA(R1, R2, KC, RAD, MODE, PART, STATE)                                                   \
    {{R1, R2, KC, RAD, MODE, PART, STATE},                                                           \
     &launch_mma2d<R1, R2, KC, RAD, MODE, PART, STATE>,                                              \
     MmaGeom<R1, R2, RAD, STATE>::WGH, MmaGeom<R1, R2, RAD, STATE>::ROW, 0, 0}

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

}  // namespace ss
