// 2-D stencil sweep as a structured-sparse (or dense) matrix product on
// gfx950 matrix cores, for states stored as FP32 values (split into hi + lo
// parts) or plain binary16 values (kernel template; instantiated by
// mma2d_f32.hip and mma2d_f16.hip).
//
// Same product as the planes kernel (mma2d_impl.hpp): one output tile of
// r2 x r1 points is y = A'' * b'', A'' the permuted staircase coefficient
// matrix and b'' the tile's halo'd patch gathered in the same K order (paper
// Sections 3.1-3.3), sixteen tiles forming the N dimension of one MMA.  What
// differs is how the patch reaches the B registers:
//  * a work item's rows arrive by LDS DMA in a staging slab as stored;
//  * one pass over the slab splits every horizontal pair of FP32 values once
//    into its packed hi and lo words (or, for binary16, moves the pair's
//    word) and writes them, side by side, into a converted slab whose row
//    gaps put the 16 tiles of a unit in 16 different LDS banks (ConvGeom);
//  * each gather is then one 8-byte (FP32 split) or 4-byte (binary16) LDS
//    read from an address fixed for the whole launch.
// With two staging slabs the DMA of the next two items overlaps the
// conversion and the products of the current one.
//
// FP32 split: three products hi*hi + hi*lo + lo*hi accumulate in FP32 (the
// lo parts carry the scale sigma, divided out at the end).  Binary16: one
// product of the binary16 coefficients and state, FP32 accumulation, the
// result rounded to binary16.
#pragma once

#include "mma2d_impl.hpp"

namespace ss {

// Per-workgroup pipeline of the converted kernels.  VMEM operations per wave
// and item: D loads (16-byte pieces, or 4-byte values when FP32 rows are not
// 16-byte aligned) and M stores.
template <int R1, int R2, int RAD, int STATE, bool VEC>
struct CPipe {
    using C = ConvGeom<R1, R2, RAD, STATE>;
    using G = typename C::G;
    static constexpr int NELEM = VEC ? C::NPIECE : C::SROWS * C::SPITCH;   // transfers per item
    static constexpr int D = (NELEM + kThreads - 1) / kThreads;
    static_assert(D * kThreads * (VEC ? 16 : 4) <= C::STAGE_ALLOC, "rounds overrun the staging room");
    static constexpr int STORES_PER_MB = (STATE == kStateF16 || VEC) ? 1 : 4;
    static constexpr int M = G::U * G::MB * STORES_PER_MB;
    // VMEM operations issued after item s's loads when it is consumed: the
    // loads of the NSLAB-1 items issued after it and the stores of the items
    // computed since (at most NSLAB)
    template <int S>
    static constexpr int W = (C::NSLAB - 1) * D + (S < C::NSLAB ? S : C::NSLAB) * M;
};

// Issue the LDS DMA of one work item into a staging slab: every row of the
// slab (SPITCH values from X0 - CH) in 16-byte pieces (or 4-byte values),
// the slab taken as one flat array so that each 64-lane transfer fills 64
// consecutive pieces.  Rows or pieces outside a zero-halo grid read from a
// zero page; pieces never straddle the grid's edge (rows are a multiple of
// CH values on this path).  Every wave issues exactly D transfers per item
// with all lanes active (the explicit waits count on it): the lanes past the
// slab's last piece copy the zero page into the room after the slab.
template <int R1, int R2, int RAD, int STATE, bool VEC, int BC>
__device__ inline void issue_staged(const void *zero_block, const MmaJob &g, char *stage, int X0, int Y0) {
    using C = ConvGeom<R1, R2, RAD, STATE>;
    using P = CPipe<R1, R2, RAD, STATE, VEC>;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    X0 = __builtin_amdgcn_readfirstlane(X0);
    Y0 = __builtin_amdgcn_readfirstlane(Y0);
    const char *zeros = static_cast<const char *>(zero_block);
    const char *in = static_cast<const char *>(g.in);
    const unsigned base = lds_addr_of(stage);
#pragma unroll
    for (int o = 0; o < P::D; ++o) {
        const int e0 = (o * kWaves + wave) * 64;      // first transfer of the instruction
        const int e = e0 + lane;
        const int per_row = VEC ? C::PIECES : C::SPITCH;
        const int r = e / per_row, c = e % per_row;
        const int gy = wrap<BC>(Y0 - RAD + r, g.ny);
        const int gx = wrap<BC>(X0 - C::CH + (VEC ? c * C::CH : c), g.nx);
        const bool ok = e < P::NELEM && (BC != kBcZero || (gy >= 0 && gy < g.ny && gx >= 0 && gx < g.nx));
        const char *src = ok ? in + ((size_t)gy * g.nx + gx) * C::EB : zeros + (VEC ? 16 : 4) * lane;
        if constexpr (VEC)
            lds_dma16(src, base + e0 * 16);
        else
            lds_dma4(src, base + e0 * 4);
    }
}

// The stored pair of staging row r whose first value is pair j's: two FP32
// values, or the word of two binary16 values (assembled from the two words
// around it when the pair starts at an odd column).
template <int R1, int R2, int RAD, int STATE>
struct StagedPair {
    float x0, x1;
    unsigned w;
};

template <int R1, int R2, int RAD, int STATE>
__device__ inline StagedPair<R1, R2, RAD, STATE> load_pair(const char *stage, int r, int j) {
    using C = ConvGeom<R1, R2, RAD, STATE>;
    const int col = r * C::SPITCH + C::P0 + 2 * j;
    StagedPair<R1, R2, RAD, STATE> v{0.f, 0.f, 0u};
    if constexpr (STATE == kStateF16) {
        if constexpr (C::P0 % 2 == 0) {
            v.w = *reinterpret_cast<const unsigned *>(stage + 2 * col);
        } else {
            const unsigned *s = reinterpret_cast<const unsigned *>(stage + 2 * (col - 1));
            v.w = __builtin_amdgcn_alignbyte(s[1], s[0], 2);
        }
    } else {
        const float *s = reinterpret_cast<const float *>(stage) + col;
        v.x0 = s[0];
        v.x1 = s[1];
    }
    return v;
}

// Write pair j of row r of the converted slab: the packed hi and lo words of
// an FP32 pair, or the binary16 word as it is.
template <int R1, int R2, int RAD, int STATE, int PART>
__device__ inline void store_pair(char *conv, int r, int j, const StagedPair<R1, R2, RAD, STATE> &v, float sigma) {
    using C = ConvGeom<R1, R2, RAD, STATE>;
    char *dst = conv + 4 * (r * C::ROWC + C::pos(j));
    if constexpr (STATE == kStateF16) {
        *reinterpret_cast<unsigned *>(dst) = v.w;
    } else {
        unsigned hi, lo;
        split2<PART>(v.x0, v.x1, sigma, &hi, &lo);
        *reinterpret_cast<u2v *>(dst) = u2v{hi, lo};
    }
}

// Convert a whole staging slab: threads own pair column t % 128 of rows
// t / 128, t / 128 + 4, ...; the RAD pairs past column 128 of each row go
// to the first SROWS * RAD threads.  All of a thread's reads are issued
// before its first write (the compiler cannot tell that the two slabs do not
// overlap, and would otherwise wait for every read in turn).
template <int R1, int R2, int RAD, int STATE, int PART>
__device__ inline void convert_item(const char *stage, char *conv, float sigma) {
    using C = ConvGeom<R1, R2, RAD, STATE>;
    using V = StagedPair<R1, R2, RAD, STATE>;
    static_assert(kThreads == 512 && C::NPAIR >= 128, "conversion thread map");
    constexpr int NI = (C::SROWS + 3) / 4;
    const int t = threadIdx.x;
    const int j = t & 127, ph = t >> 7;
    const bool extra = t < C::SROWS * RAD;
    const int er = t / RAD, ej = 128 + t % RAD;
    V v[NI], ev{};
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int r = ph + 4 * i;
        if (4 * i + 3 < C::SROWS || r < C::SROWS) v[i] = load_pair<R1, R2, RAD, STATE>(stage, r, j);
    }
    if (extra) ev = load_pair<R1, R2, RAD, STATE>(stage, er, ej);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int r = ph + 4 * i;
        if (4 * i + 3 < C::SROWS || r < C::SROWS) store_pair<R1, R2, RAD, STATE, PART>(conv, r, j, v[i], sigma);
    }
    if (extra) store_pair<R1, R2, RAD, STATE, PART>(conv, er, ej, ev, sigma);
}

// Gather addresses of a lane: one 32-bit word per B register, or, where
// that would take too many registers (32 and more), two 16-bit addresses per
// word (a converted slab is smaller than 64 KiB), unpacked at each use.  The
// packed word passes through an empty asm that takes a loop-varying value,
// so that the unpacked addresses are not hoisted out of the item loop and
// kept live (which would undo the packing).
template <int KC, int VPK>
struct GatherAddr {
    static constexpr bool PACK = KC * VPK >= 32;
    unsigned w[KC][PACK ? VPK / 2 : VPK];
    __device__ inline void set(int kc, int v, unsigned a) {
        if constexpr (PACK)
            w[kc][v >> 1] = (v & 1) ? (w[kc][v >> 1] | (a << 16)) : a;
        else
            w[kc][v] = a;
    }
    __device__ inline unsigned get(int kc, int v, int salt) const {
        if constexpr (PACK) {
            unsigned x = w[kc][v >> 1];
            asm("" : "+v"(x) : "s"(salt));
            return (v & 1) ? (x >> 16) : (x & 0xffffu);
        } else {
            return w[kc][v];
        }
    }
};

// Multiply one work item out of the converted slab and write its outputs.
// Wave w owns units (w / NCOLS) * U + u of unit column w % NCOLS; gaddr holds
// the lane's gather addresses (bytes from the slab) for unit 0.
template <int R1, int R2, int KC, int RAD, int MODE, int PART, int STATE, bool VEC>
__device__ inline void compute_conv(float inv_sigma, const MmaJob &g, const char *conv,
                                    const uint4 (&ahi)[R1 * R2 / 16][KC], const uint4 (&alo)[R1 * R2 / 16][KC],
                                    const unsigned (&aidx)[R1 * R2 / 16][KC],
                                    const GatherAddr<KC, (MODE == kSparse) ? 8 : 4> &gaddr, int X0, int Y0,
                                    int salt) {
    using C = ConvGeom<R1, R2, RAD, STATE>;
    using G = typename C::G;
    constexpr int MB = G::MB;
    constexpr int VPK = (MODE == kSparse) ? 8 : 4;
    constexpr bool SPLIT = STATE == kStateF32;
    // with four or more M-blocks between them, hi*lo and lo*hi of one block
    // can share an accumulator without back-to-back dependent products
    constexpr bool MERGE = MB >= 4;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nb = wave / G::NCOLS;
    const int nbc = wave % G::NCOLS;
    const int n = lane & 15;
    const int q = lane >> 4;
    const int tx_t = n % G::NBX;
    const int ty_t = n / G::NBX;
    X0 = __builtin_amdgcn_readfirstlane(X0);
    Y0 = __builtin_amdgcn_readfirstlane(Y0);
    const int rows_left = min(G::WGH, g.ny - Y0);
    const int xbase = X0 + nbc * G::UW + tx_t * R1;
#pragma unroll
    for (int u = 0; u < G::U; ++u) {
        const int uoff = u * G::NBH * C::ROWC * 4;      // unit u's rows below unit 0's
        const int srow0 = (nb * G::U + u) * G::NBH + ty_t * R2;
        f4 accm[MB], acc1[MB], acc2[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            accm[mb] = f4{0.f, 0.f, 0.f, 0.f};
            acc1[mb] = f4{0.f, 0.f, 0.f, 0.f};
            acc2[mb] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            unsigned bh[VPK], bl[VPK];
#pragma unroll
            for (int v = 0; v < VPK; ++v) {
                const char *a = conv + gaddr.get(kc, v, salt + u) + uoff;
                if constexpr (SPLIT) {
                    const u2v w = *reinterpret_cast<const u2v *>(a);
                    bh[v] = w.x;
                    bl[v] = w.y;
                } else {
                    bh[v] = *reinterpret_cast<const unsigned *>(a);
                    bl[v] = 0;
                }
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) accm[mb] = mma<MODE, PART>(ahi[mb][kc], bh, accm[mb], aidx[mb][kc]);
            if constexpr (SPLIT) {
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) acc1[mb] = mma<MODE, PART>(ahi[mb][kc], bl, acc1[mb], aidx[mb][kc]);
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    if constexpr (MERGE)
                        acc1[mb] = mma<MODE, PART>(alo[mb][kc], bh, acc1[mb], aidx[mb][kc]);
                    else
                        acc2[mb] = mma<MODE, PART>(alo[mb][kc], bh, acc2[mb], aidx[mb][kc]);
                }
            }
        }
        // write back: accumulator rows 4q..4q+3 of M-block mb are outputs
        // mb*16 + 4q + i of the tile, four consecutive x positions; buffer
        // stores with an out-of-range offset drop the write
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int o = mb * 16 + 4 * q;
            const int gyr = srow0 + o / R1;
            const int gx = xbase + o % R1;
            const bool row_ok = gyr < rows_left;
            float ys[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if constexpr (!SPLIT)
                    ys[i] = accm[mb][i];
                else if constexpr (MERGE)
                    ys[i] = accm[mb][i] + acc1[mb][i] * inv_sigma;
                else
                    ys[i] = accm[mb][i] + (acc1[mb][i] + acc2[mb][i]) * inv_sigma;
            }
            if constexpr (STATE == kStateF16) {
                // round to binary16 (nearest even); rows are a multiple of 8
                // values, so the four outputs are all in or all out
                const h2v p0 = __builtin_convertvector((f2v{ys[0], ys[1]}), h2v);
                const h2v p1 = __builtin_convertvector((f2v{ys[2], ys[3]}), h2v);
                const u2v hv = {__builtin_bit_cast(unsigned, p0), __builtin_bit_cast(unsigned, p1)};
                unsigned short *out = static_cast<unsigned short *>(g.out);
                const __amdgpu_buffer_rsrc_t rs = uniform_rsrc(out + (size_t)Y0 * g.nx, rows_left * g.nx * 2);
                const unsigned o2 = row_ok && gx < g.nx ? (unsigned)(gyr * g.nx + gx) * 2u : kOob;
                __builtin_amdgcn_raw_buffer_store_b64(hv, rs, o2, 0, 0);
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

// Persistent sweep kernel, one workgroup per CU, with the work-item order and
// XCD mapping of k_mma2d.  Per item s: wait for its staging slab, convert it
// (the converted slab is free: every wave has finished item s-1), then
// refill the staging slab with item s+2 and multiply item s out.
template <int R1, int R2, int KC, int RAD, int MODE, int PART, int STATE, bool VEC, int BC>
__global__ __launch_bounds__(kThreads, 1) void k_mma2c(MmaArgs p) {
    using C = ConvGeom<R1, R2, RAD, STATE>;
    using G = typename C::G;
    using P = CPipe<R1, R2, RAD, STATE, VEC>;
    constexpr int MB = G::MB;
    constexpr int VPK = (MODE == kSparse) ? 8 : 4;
    constexpr int NS = C::NSLAB;
    __shared__ __attribute__((aligned(16))) char lds[C::LDS_BYTES];
    char *conv = lds;
    auto stage = [&](int i) { return lds + C::CONV_BYTES + i * C::STAGE_ALLOC; };

    const float sigma = 1.0f / p.inv_sigma;
    const float inv_sigma = p.inv_sigma;
    const int nxcd = p.nxcd;
    const int nwg = gridDim.x;
    const int xcd = blockIdx.x % nxcd;
    const int stride = nwg / nxcd + (xcd < nwg % nxcd ? 1 : 0);
    const int before = xcd * (nwg / nxcd) + min(xcd, nwg % nxcd);
    const int range_begin = (int)((long long)p.total_items * before / nwg);
    const int total = (int)((long long)p.total_items * (before + stride) / nwg);
    const int first = range_begin + blockIdx.x / nxcd;
    if (first >= total) return;

    // gather addresses of unit 0: the tile's patch origin in the converted
    // slab plus the plan's offset of each B register
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4;
    GatherAddr<KC, VPK> gaddr;
    static_assert(!GatherAddr<KC, VPK>::PACK || C::CONV_BYTES <= 65536, "16-bit gather addresses");
    {
        const int wave = threadIdx.x >> 6;
        const int n = lane & 15;
        const int srow0 = (wave / G::NCOLS) * G::U * G::NBH + (n / G::NBX) * R2;
        const int pair0 = ((wave % G::NCOLS) * G::UW + (n % G::NBX) * R1) / 2;
        const int tile = 4 * (srow0 * C::ROWC + C::pos(pair0));
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int v = 0; v < VPK; ++v) gaddr.set(kc, v, (unsigned)(tile + p.boff[(kc * 4 + q) * VPK + v]));
    }
    uint4 ahi[MB][KC], alo[MB][KC];
    unsigned aidx[MB][KC];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const int t = (mb * KC + kc) * 64 + lane;
            ahi[mb][kc] = p.a_hi[t];
            alo[mb][kc] = STATE == kStateF32 ? p.a_lo[t] : uint4{0u, 0u, 0u, 0u};
            aidx[mb][kc] = (MODE == kSparse) ? p.a_idx[t] : 0u;
        }
    wait_vmcnt<0>();

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
        const MmaJob g = p.job[j];
        issue_staged<R1, R2, RAD, STATE, VEC, BC>(p.zeros, g, stage(s % NS), X0, Y0);
    };
#pragma unroll
    for (int s = 0; s < NS; ++s) issue(s);

#pragma unroll 1
    for (int s = 0;; ++s) {
        switch (s) {
            case 0: wait_vmcnt<P::template W<0>>(); break;
            case 1: wait_vmcnt<P::template W<1>>(); break;
            default: wait_vmcnt<P::template W<2>>(); break;
        }
        __builtin_amdgcn_s_barrier();
        convert_item<R1, R2, RAD, STATE, PART>(stage(s % NS), conv, sigma);
        __builtin_amdgcn_s_waitcnt(0xC07F);          // lgkmcnt(0): converted pairs written
        __builtin_amdgcn_s_barrier();
        issue(s + NS);
        int j, X0, Y0;
        locate(item(s), j, X0, Y0);
        const MmaJob g = p.job[j];
        compute_conv<R1, R2, KC, RAD, MODE, PART, STATE, VEC>(inv_sigma, g, conv, ahi, alo, aidx, gaddr, X0, Y0,
                                                              s * G::U);
        if (first + (s + 1) * stride >= total) break;
    }
    // the pipeline always runs NS items ahead: let those transfers land
    // before the workgroup's LDS is released
    wait_vmcnt<0>();
}

template <int R1, int R2, int KC, int RAD, int MODE, int PART, int STATE, bool VEC, int BC>
static hipError_t launch_c_bc(const MmaArgs &a, hipStream_t s) {
    int cus = 0, xcds = 0;
    if (const hipError_t e = device_shape(&cus, &xcds); e != hipSuccess) return e;
    MmaArgs b = a;
    b.nxcd = xcds;
    const int g = a.total_items < cus ? a.total_items : cus;
    hipLaunchKernelGGL((k_mma2c<R1, R2, KC, RAD, MODE, PART, STATE, VEC, BC>), dim3(g), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

// Number the jobs' work items, then pick the variant every job of the launch
// can use: 16-byte pieces or 4-byte values (FP32 rows that are not a multiple
// of 4 values), and the cheapest boundary handling valid for all of them.
// Binary16 rows must be a multiple of 8 values (the planner checks).
template <int R1, int R2, int KC, int RAD, int MODE, int PART, int STATE>
static hipError_t launch_mma2c(MmaArgs &a, hipStream_t s) {
    using C = ConvGeom<R1, R2, RAD, STATE>;
    using G = typename C::G;
    if (a.njobs < 1 || a.njobs > kMaxJobs) return hipErrorInvalidValue;
    int items = 0;
    bool vec = true, wrap1 = true;
    for (int j = 0; j < a.njobs; ++j) {
        const MmaJob &g = a.job[j];
        a.job[j].item0 = items;
        items += ((g.nx + kBandX - 1) / kBandX) * ((g.ny + G::WGH - 1) / G::WGH);
        vec = vec && (g.nx % C::CH) == 0;
        // one wrap suffices when every index is within one grid length
        wrap1 = wrap1 && g.ny >= G::SROWS && g.nx >= C::SPITCH;
    }
    a.total_items = items;
    if (items == 0) return hipSuccess;
    if constexpr (STATE == kStateF16) {
        if (!vec) return hipErrorInvalidValue;
        if (!a.periodic) return launch_c_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcZero>(a, s);
        if (wrap1) return launch_c_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcWrap1>(a, s);
        return launch_c_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcWrapN>(a, s);
    } else {
        if (vec) {
            if (!a.periodic) return launch_c_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcZero>(a, s);
            if (wrap1) return launch_c_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcWrap1>(a, s);
            return launch_c_bc<R1, R2, KC, RAD, MODE, PART, STATE, true, kBcWrapN>(a, s);
        }
        if (!a.periodic) return launch_c_bc<R1, R2, KC, RAD, MODE, PART, STATE, false, kBcZero>(a, s);
        if (wrap1) return launch_c_bc<R1, R2, KC, RAD, MODE, PART, STATE, false, kBcWrap1>(a, s);
        return launch_c_bc<R1, R2, KC, RAD, MODE, PART, STATE, false, kBcWrapN>(a, s);
    }
}

#define SS_MMA_CONV(R1, R2, KC, RAD, MODE, PART, STATE)                                                         \
    {{R1, R2, KC, RAD, MODE, PART, STATE},                                                                      \
     &launch_mma2c<R1, R2, KC, RAD, MODE, PART, STATE>,                                                         \
     MmaGeom<R1, R2, RAD, kStateF32>::WGH, ConvGeom<R1, R2, RAD, STATE>::ROWC,                                  \
     ConvGeom<R1, R2, RAD, STATE>::PW, ConvGeom<R1, R2, RAD, STATE>::PADG}

}  // namespace ss
