// 2-D stencil sweep as a structured-sparse (or dense) matrix product on
// gfx950 matrix cores.
//
// One output tile of r2 x r1 points is y = A'' * b'' where A'' (m' x K) is the
// permuted staircase coefficient matrix and b'' the tile's halo'd input patch
// gathered in the same K order (paper Sections 3.1-3.3).  Sixteen tiles form
// the N dimension of one MMA.  The FP32 state is staged into LDS as is and
// split into hi + lo parts as it is gathered into B registers; three products
// hi*hi + hi*lo + lo*hi accumulate in FP32 (the lo parts carry a scale sigma
// that is divided out at the end).
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
// read feeds one hi register and one lo register.
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

// Split two FP32 values into packed hi parts and sigma-scaled lo parts.
template <int PART>
__device__ inline void split2(float x0, float x1, float sigma, unsigned *hi, unsigned *lo) {
    if constexpr (PART == kPartF16) {
        const _Float16 h0 = (_Float16)x0, h1 = (_Float16)x1;
        const _Float16 l0 = (_Float16)((x0 - (float)h0) * sigma);
        const _Float16 l1 = (_Float16)((x1 - (float)h1) * sigma);
        *hi = (unsigned)__builtin_bit_cast(unsigned short, h0) |
              ((unsigned)__builtin_bit_cast(unsigned short, h1) << 16);
        *lo = (unsigned)__builtin_bit_cast(unsigned short, l0) |
              ((unsigned)__builtin_bit_cast(unsigned short, l1) << 16);
    } else {
        const __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1;
        const __bf16 l0 = (__bf16)((x0 - (float)h0) * sigma);
        const __bf16 l1 = (__bf16)((x1 - (float)h1) * sigma);
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

// Raw buffer descriptor word 3 for gfx9-family (gfx950) and an offset past
// any descriptor's range (out-of-range buffer stores are dropped).
constexpr int kRsrcWord3 = 0x00020000;
constexpr unsigned kOob = 0x80000000u;

typedef __attribute__((address_space(3))) void lds_void;

// Buffer descriptor over `bytes` bytes at `base` (wave-uniform values, read
// from lane 0 so that the descriptor is known to live in scalar registers).
__device__ inline __amdgpu_buffer_rsrc_t uniform_rsrc(float *base, int bytes) {
    const unsigned long long b = (unsigned long long)base;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    float *ub = (float *)(((unsigned long long)hi << 32) | lo);
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
// A wave never has more than 63 VMEM operations outstanding (issue stalls
// first), so a wait for an operation followed by 63 or more is a no-op.
template <int N>
__device__ inline void wait_vmcnt() {
    static_assert(N >= 0, "vmcnt range");
    constexpr int C = N < 63 ? N : 63;
    __builtin_amdgcn_s_waitcnt((C & 15) | ((C >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Per-workgroup pipeline geometry of the 2-D MMA kernel.
template <int R1, int R2, int RAD, bool VEC>
struct Pipe {
    using G = MmaGeom<R1, R2, RAD>;
    static constexpr int DRW = (G::SROWS + kWaves - 1) / kWaves;      // slab rows each wave loads
    static constexpr int DMA_PER_ROW = VEC ? 1 : kBandX / 64;         // LDS-DMA ops per row
    static constexpr int NHALO = G::SROWS * 2 * RAD;                   // halo columns of a slab
    static constexpr int HOPS = (NHALO + 64 * kWaves - 1) / (64 * kWaves);  // halo DMA ops per wave
    static constexpr int HSTRIP = HOPS * 64 * kWaves;                  // halo staging floats per slab
    static constexpr int D = DRW * DMA_PER_ROW + HOPS;                  // VMEM loads per wave per item
    static constexpr int M = VEC ? G::MB : 4 * G::MB;                   // VMEM stores per wave per item
    // VMEM operations issued after an item's last load when its slab is
    // consumed at pipeline step s: two later items' loads and min(s, 3)
    // items' stores
    static constexpr int W0 = 2 * D, W1 = 2 * D + M, W2 = 2 * D + 2 * M, W3 = 2 * D + 3 * M;
};

// LDS DMA: each active lane copies 16 (or 4) bytes from its global address to
// LDS at lds_addr + 16*lane (or 4*lane).  Written as inline assembly so that
// the compiler does not track these transfers: the pipeline waits for them
// explicitly with s_waitcnt vmcnt before the barrier that publishes a slab.
__device__ inline void lds_dma16(const void *src, unsigned lds_addr) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(src), "s"(lds_addr)
                 : "memory", "m0");
}
__device__ inline void lds_dma4(const void *src, unsigned lds_addr) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %0, off"
                 :
                 : "v"(src), "s"(lds_addr)
                 : "memory", "m0");
}
__device__ inline unsigned lds_addr_of(const float *p) {
    return (unsigned)(size_t)(const __attribute__((address_space(3))) float *)p;
}

// Issue the loads of one work item: the 256 interior columns of every slab
// row (one 64-lane 16-byte transfer per row, or four 64-lane 4-byte transfers
// when rows are not 16-byte aligned) into the slab, and the 2*RAD halo
// columns of every row into a staging strip (put_halo moves them into place).
// Rows or columns outside a zero-halo grid read from a zero page.  Every wave
// issues the same number of transfers for every item (item and row indices
// are clamped), which is what the explicit waits count on.
template <int R1, int R2, int RAD, bool VEC, int BC>
__device__ inline void issue_item(const MmaArgs &p, const MmaJob &g, float *slab, float *strip, int X0, int Y0) {
    using G = MmaGeom<R1, R2, RAD>;
    using P = Pipe<R1, R2, RAD, VEC>;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    X0 = __builtin_amdgcn_readfirstlane(X0);
    Y0 = __builtin_amdgcn_readfirstlane(Y0);
#pragma unroll
    for (int d = 0; d < P::DRW; ++d) {
        const int r = min(wave + d * kWaves, G::SROWS - 1);
        const int gy = wrap<BC>(Y0 - RAD + r, g.ny);
        const bool row_ok = BC != kBcZero || (gy >= 0 && gy < g.ny);
        const unsigned dst = lds_addr_of(slab + r * G::CPITCH + G::HL);
        if constexpr (VEC) {
            const int gx = wrap<BC>(X0 + 4 * lane, g.nx);
            const bool ok = BC != kBcZero || (row_ok && gx < g.nx);
            const float *src = ok ? g.in + (size_t)gy * g.nx + gx : p.zeros + 4 * lane;
            lds_dma16(src, dst);
        } else {
#pragma unroll
            for (int h = 0; h < P::DMA_PER_ROW; ++h) {
                const int gx = wrap<BC>(X0 + 64 * h + lane, g.nx);
                const bool ok = BC != kBcZero || (row_ok && gx < g.nx);
                const float *src = ok ? g.in + (size_t)gy * g.nx + gx : p.zeros + lane;
                lds_dma4(src, dst + 256 * h);
            }
        }
    }
#pragma unroll
    for (int h = 0; h < P::HOPS; ++h) {
        const int base = (h * kWaves + wave) * 64;
        const int e = min(base + lane, P::NHALO - 1);
        const int r = e / (2 * RAD), j = e % (2 * RAD);
        const int gy = wrap<BC>(Y0 - RAD + r, g.ny);
        const int gx = wrap<BC>(j < RAD ? X0 - RAD + j : X0 + kBandX + (j - RAD), g.nx);
        const bool ok = BC != kBcZero || (gy >= 0 && gy < g.ny && gx >= 0 && gx < g.nx);
        const float *src = ok ? g.in + (size_t)gy * g.nx + gx : p.zeros + lane;
        lds_dma4(src, lds_addr_of(strip + base));
    }
}

// Move an item's halo columns from the staging strip into the slab.
template <int R1, int R2, int RAD, bool VEC>
__device__ inline void put_halo(float *slab, const float *strip) {
    using G = MmaGeom<R1, R2, RAD>;
    using P = Pipe<R1, R2, RAD, VEC>;
    for (int e = threadIdx.x; e < P::NHALO; e += kThreads) {
        const int r = e / (2 * RAD), j = e % (2 * RAD);
        const int c = j < RAD ? G::HL - RAD + j : G::HL + kBandX + (j - RAD);
        slab[r * G::CPITCH + c] = strip[e];
    }
}

// Multiply one work item out of its LDS slab and write its outputs.  Wave w
// owns N-block w: 16 tiles of R2 x R1 outputs.
template <int R1, int R2, int KC, int RAD, int MODE, int PART, bool VEC>
__device__ inline void compute_item(const MmaArgs &p, const MmaJob &g, const float *slab, const uint4 (&ahi)[R1 * R2 / 16][KC],
                                    const uint4 (&alo)[R1 * R2 / 16][KC], const unsigned (&aidx)[R1 * R2 / 16][KC],
                                    const int (&off)[KC][(MODE == kSparse) ? 8 : 4], int X0, int Y0, float sigma) {
    using G = MmaGeom<R1, R2, RAD>;
    constexpr int MB = G::MB;
    constexpr int VPK = (MODE == kSparse) ? 8 : 4;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nb = wave / kNbCols;            // N-block row of the item
    const int nbc = wave % kNbCols;           // N-block column of the band
    const int n = lane & 15;
    const int q = lane >> 4;
    const int tx_t = n % G::NBX;
    const int ty_t = n / G::NBX;
    // X0, Y0 are uniform; saying so keeps the store descriptor in SGPRs
    X0 = __builtin_amdgcn_readfirstlane(X0);
    Y0 = __builtin_amdgcn_readfirstlane(Y0);
    const int rows_left = min(G::WGH, g.ny - Y0);
    const __amdgpu_buffer_rsrc_t orsrc = uniform_rsrc(g.out + (size_t)Y0 * g.nx, rows_left * g.nx * 4);
    const int srow0 = nb * G::NBH + ty_t * R2;
    const float *tb = slab + srow0 * G::CPITCH + (G::HL - RAD) + nbc * 128 + tx_t * R1;
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
            const float *src = tb + off[kc][v];
            split2<PART>(src[0], src[1], sigma, &bh[v], &bl[v]);
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            accm[mb] = mma<MODE, PART>(ahi[mb][kc], bh, accm[mb], aidx[mb][kc]);
            accc[mb] = mma<MODE, PART>(ahi[mb][kc], bl, accc[mb], aidx[mb][kc]);
            accc[mb] = mma<MODE, PART>(alo[mb][kc], bh, accc[mb], aidx[mb][kc]);
        }
    }
    // write back: accumulator rows 4q..4q+3 of M-block mb are outputs
    // mb*16 + 4q + i of the tile, four consecutive x positions.  Buffer stores
    // with an out-of-range offset drop the write, so every store is issued.
    const int yrel = nb * G::NBH + ty_t * R2;
    const int xbase = X0 + nbc * 128 + tx_t * R1;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int o = mb * 16 + 4 * q;
        const int gyr = yrel + o / R1;
        const int gx = xbase + o % R1;
        f4 y;
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] = accm[mb][i] + accc[mb][i] * p.inv_sigma;
        const bool row_ok = gyr < rows_left;
        if constexpr (VEC) {
            const unsigned o4 = row_ok && gx < g.nx ? (unsigned)(gyr * g.nx + gx) * 4u : kOob;
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, y), orsrc, o4, 0, 0);
        } else {
            // one scalar per store: the element is copied out of the vector
            // before its bits are reinterpreted
            const float ys[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const unsigned o1 = row_ok && gx + i < g.nx ? (unsigned)(gyr * g.nx + gx + i) * 4u : kOob;
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(ys[i]), orsrc, o1, 0, 0);
            }
        }
    }
}

// Persistent sweep kernel, one workgroup per CU.  Work items are (256-column
// band, WGH-row block) pairs in row-block-major order; workgroup g takes
// items g, g + G, g + 2G, ... so that at any time the device works on a
// contiguous strip of rows.  Four LDS slabs rotate: while item s is
// multiplied out of one, the inputs of items s+1..s+3 stream into the others
// by LDS DMA, which keeps about 100 KB per CU in flight without holding it in
// registers.
template <int R1, int R2, int KC, int RAD, int MODE, int PART, bool VEC, int BC>
__global__ __launch_bounds__(kThreads, 1) void k_mma2d(MmaArgs p) {
    using G = MmaGeom<R1, R2, RAD>;
    using P = Pipe<R1, R2, RAD, VEC>;
    constexpr int MB = G::MB;
    constexpr int VPK = (MODE == kSparse) ? 8 : 4;  // B registers per K chunk
    __shared__ float S0[G::SLAB_F];
    __shared__ float S1[G::SLAB_F];
    __shared__ float S2[G::SLAB_F];
    __shared__ float S3[G::SLAB_F];
    __shared__ float H0[P::HSTRIP];
    __shared__ float H1[P::HSTRIP];
    __shared__ float H2[P::HSTRIP];
    __shared__ float H3[P::HSTRIP];

    const float sigma = 1.0f / p.inv_sigma;
    // Workgroups are dealt to the XCDs round robin (workgroup g runs on XCD
    // g mod X).  Each XCD takes one contiguous range of items, in proportion
    // to its workgroup count, and its workgroups interleave over that range:
    // the rows an item shares with its neighbours (halo columns and rows)
    // are then fetched into the same L2 at about the same time.
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
    auto issue = [&](int s, float *slab, float *strip) {
        int j, X0, Y0;
        locate(item(s), j, X0, Y0);
        issue_item<R1, R2, RAD, VEC, BC>(p, p.job[j], slab, strip, X0, Y0);
    };
    issue(0, S0, H0);
    issue(1, S1, H1);
    issue(2, S2, H2);

    // one pipeline step: wait for slab `cur` (item s), publish it, refill
    // slab `nxt` (consumed at step s-1) with item s+3, multiply item s
    auto step = [&](int s, float *cur, float *hcur, float *nxt, float *hnxt) {
        if (s == 0) wait_vmcnt<P::W0>();
        else if (s == 1) wait_vmcnt<P::W1>();
        else if (s == 2) wait_vmcnt<P::W2>();
        else wait_vmcnt<P::W3>();
        __builtin_amdgcn_s_barrier();            // every wave's transfers for item s landed
        put_halo<R1, R2, RAD, VEC>(cur, hcur);
        __builtin_amdgcn_s_waitcnt(0xC07F);      // lgkmcnt(0): halo writes done
        __builtin_amdgcn_s_barrier();
        issue(s + 3, nxt, hnxt);
        int j, X0, Y0;
        locate(item(s), j, X0, Y0);
        compute_item<R1, R2, KC, RAD, MODE, PART, VEC>(p, p.job[j], cur, ahi, alo, aidx, off, X0, Y0, sigma);
    };

#pragma unroll 1
    for (int s = 0;; s += 4) {
        step(s, S0, H0, S3, H3);
        if (first + (s + 1) * stride >= total) break;
        step(s + 1, S1, H1, S0, H0);
        if (first + (s + 2) * stride >= total) break;
        step(s + 2, S2, H2, S1, H1);
        if (first + (s + 3) * stride >= total) break;
        step(s + 3, S3, H3, S2, H2);
        if (first + (s + 4) * stride >= total) break;
    }
    // the pipeline always runs three items ahead: let those transfers land
    // before the workgroup's LDS is released
    wait_vmcnt<0>();
}

// Compute units and XCDs of the current device (queried once per device).
static hipError_t device_shape(int *cus, int *xcds) {
    constexpr int kMaxDevices = 64;
    static int cache[kMaxDevices][2];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (cache[dev][0] == 0) {
        int c = 0, x = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipDeviceGetAttribute(&x, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || c < 1)
            return hipErrorInvalidDevice;
        cache[dev][1] = x > 0 ? x : 1;
        cache[dev][0] = c;
    }
    *cus = cache[dev][0];
    *xcds = cache[dev][1];
    return hipSuccess;
}

template <int R1, int R2, int KC, int RAD, int MODE, int PART, bool VEC, int BC>
static hipError_t launch_bc(const MmaArgs &a, hipStream_t s) {
    int cus = 0, xcds = 0;
    if (const hipError_t e = device_shape(&cus, &xcds); e != hipSuccess) return e;
    MmaArgs b = a;
    b.nxcd = xcds;
    // one workgroup per CU, never more workgroups than items
    const int g = a.total_items < cus ? a.total_items : cus;
    hipLaunchKernelGGL((k_mma2d<R1, R2, KC, RAD, MODE, PART, VEC, BC>), dim3(g), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

// Number the jobs' work items, then pick the kernel variant every job of the
// launch can use: 16-byte-aligned rows or not, and the cheapest boundary
// handling valid for all of them.
template <int R1, int R2, int KC, int RAD, int MODE, int PART>
static hipError_t launch_mma2d(MmaArgs &a, hipStream_t s) {
    using G = MmaGeom<R1, R2, RAD>;
    if (a.njobs < 1 || a.njobs > kMaxJobs) return hipErrorInvalidValue;
    int items = 0;
    bool vec = true, wrap1 = true;
    for (int j = 0; j < a.njobs; ++j) {
        const MmaJob &g = a.job[j];
        a.job[j].item0 = items;
        items += ((g.nx + kBandX - 1) / kBandX) * ((g.ny + G::WGH - 1) / G::WGH);
        vec = vec && (g.nx & 3) == 0;
        // one wrap suffices when every index is within one grid length
        wrap1 = wrap1 && g.ny >= G::SROWS && g.nx >= kBandX + 2 * RAD;
    }
    a.total_items = items;
    if (items == 0) return hipSuccess;
    if (vec) {
        if (!a.periodic) return launch_bc<R1, R2, KC, RAD, MODE, PART, true, kBcZero>(a, s);
        if (wrap1) return launch_bc<R1, R2, KC, RAD, MODE, PART, true, kBcWrap1>(a, s);
        return launch_bc<R1, R2, KC, RAD, MODE, PART, true, kBcWrapN>(a, s);
    }
    if (!a.periodic) return launch_bc<R1, R2, KC, RAD, MODE, PART, false, kBcZero>(a, s);
    if (wrap1) return launch_bc<R1, R2, KC, RAD, MODE, PART, false, kBcWrap1>(a, s);
    return launch_bc<R1, R2, KC, RAD, MODE, PART, false, kBcWrapN>(a, s);
}

struct MmaEntry {
    MmaKey key;
    MmaLaunch fn;
    int wgh, cpitch;
};

#define SS_MMA(R1, R2, KC, RAD, MODE, PART)                                                         \
    {{R1, R2, KC, RAD, MODE, PART},                                                                 \
     &launch_mma2d<R1, R2, KC, RAD, MODE, PART>,                                                    \
     MmaGeom<R1, R2, RAD>::WGH, MmaGeom<R1, R2, RAD>::CPITCH}

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

bool mma2d_geometry(const MmaKey &k, int *wgh, int *cpitch) {
    for (const auto &e : kMmaTable)
        if (e.key.r1 == k.r1 && e.key.r2 == k.r2 && e.key.kc == k.kc && e.key.rad == k.rad &&
            e.key.mode == k.mode && e.key.part == k.part) {
            *wgh = e.wgh;
            *cpitch = e.cpitch;
            return true;
        }
    return false;
}

}  // namespace ss
