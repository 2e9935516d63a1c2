// 2-D stencil sweep as a structured-sparse (or dense) matrix product on
// gfx950 matrix cores (kernel template; instantiated by mma2d_f32_r*.hip,
// mma2d_f16.hip and mma2d_planes.hip), for a state stored as FP32 values
// (split into binary16 or bfloat16 hi + lo parts), as bfloat16 hi and lo
// planes, or as plain binary16 values.
//
// One output tile of r2 x r1 points is y = A'' * b'', A'' the permuted
// staircase coefficient matrix and b'' the tile's halo'd input patch
// gathered in the same K order (paper Sections 3.1-3.3); sixteen tiles form
// the N dimension of one MMA.  The patch reaches the B registers in three
// steps:
//  * a work item's rows arrive by LDS DMA in a staging slab as stored;
//  * one pass over the slab turns every horizontal pair of values into the
//    words a B register takes -- an FP32 pair split once into its packed hi
//    and lo words, a planes pair's hi-plane and lo-plane words, a binary16
//    pair's word -- and writes them, side by side, into a converted slab
//    whose row gaps put the 16 tiles of a unit in 16 different LDS banks
//    (ConvGeom);
//  * each gather is then one 8-byte (hi and lo) or 4-byte (binary16) LDS
//    read from an address fixed for the whole launch.
// With two staging slabs the DMA of the next two items overlaps the
// conversion and the products of the current one.
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
// Split states: three products hi*hi + hi*lo + lo*hi accumulate in FP32 (the
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
    static constexpr int STORES_PER_MB =
        STATE == kStatePlanes3 ? 3 : STATE == kStatePlanes ? 2 : (STATE == kStateF16 || VEC) ? 1 : 4;
    static constexpr int M = G::U * G::MB * STORES_PER_MB;
    // VMEM operations issued after item s's loads when it is consumed: the
    // loads of the NSLAB-1 items issued after it and the stores of the items
    // computed since (at most NSLAB)
    template <int S>
    static constexpr int W = (C::NSLAB - 1) * D + (S < C::NSLAB ? S : C::NSLAB) * M;
};

// 24-bit unsigned multiplies (full-rate vector instructions; a 32-bit
// multiply takes four passes), written out so that the compiler does not
// widen them: a * b and a * b + c, b wave-uniform, all below 2^24.
__device__ inline unsigned mul_u24(unsigned a, unsigned b) {
    unsigned d;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(d) : "s"(b), "v"(a));
    return d;
}
__device__ inline unsigned mad_u24(unsigned a, unsigned b, unsigned c) {
    unsigned d;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "s"(b), "v"(c));
    return d;
}

// x / D for x < XMAX as one 24-bit multiply and a shift: M = ceil(2^S / D)
// with M * D - 2^S small enough that the truncation never reaches the next
// integer below XMAX.
template <unsigned D, unsigned XMAX>
struct DivSmall {
    static constexpr int find_shift() {
        for (int s = 0; s < 32; ++s) {
            const unsigned long long m = ((1ull << s) + D - 1) / D;
            if (m < (1ull << 24) && (XMAX - 1) * m < (1ull << 32) && (XMAX - 1) * (m * D - (1ull << s)) < (1ull << s))
                return s;
        }
        return -1;
    }
    static constexpr int S = find_shift();
    static_assert(S >= 0 && XMAX < (1u << 24), "no 24-bit multiplier for this divisor");
    static constexpr unsigned M = (unsigned)(((1ull << S) + D - 1) / D);
    // every quotient checked at compile time
    static constexpr bool exact() {
        for (unsigned long long x = 0; x < XMAX; ++x)
            if (((x * M) & 0xffffffffull) >> S != x / D) return false;
        return true;
    }
    static_assert(exact(), "24-bit division does not match");
    static __device__ inline unsigned div(unsigned x) { return mul_u24(x, M) >> S; }
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
    const unsigned base = lds_addr_of(stage);
    constexpr unsigned PER_ROW = VEC ? C::NPL * C::PIECES : C::SPITCH;   // transfers per slab row
    constexpr unsigned TB = VEC ? 16 : 4;                                  // bytes per transfer
    const unsigned long long plane_bytes = (unsigned long long)(unsigned)g.ny * (unsigned)g.nx * C::EB;
    const int sy0 = Y0 - RAD, sx0 = X0 - C::CH;     // first staged row and column
    // an item whose rows and columns all lie inside the grid (every item but
    // those along the edges) reads at 32-bit offsets from one scalar base:
    // no per-lane bounds, wrapping or 64-bit arithmetic, and only 24-bit
    // multiplies (rows shorter than 16 MiB, planes together under 2 GiB)
    const bool inside = sy0 >= 0 && sy0 + C::SROWS <= g.ny && sx0 >= 0 && sx0 + C::SPITCH <= g.nx &&
                        (unsigned long long)C::NPL * plane_bytes < (1ull << 31) &&
                        (unsigned)g.nx * C::EB < (1u << 24);
    if (inside) {
        const char *sbase = static_cast<const char *>(g.in) + ((size_t)sy0 * (unsigned)g.nx + sx0) * C::EB;
        const unsigned row_bytes = (unsigned)g.nx * C::EB;
        using DR = DivSmall<PER_ROW, P::D * kThreads>;
#pragma unroll
        for (int o = 0; o < P::D; ++o) {
            const int e0 = (o * kWaves + wave) * 64;
            const unsigned e = (unsigned)e0 + lane;
            const unsigned r = DR::div(e), cp = e - mul_u24(r, PER_ROW);
            unsigned c = cp, poff = 0;
            if constexpr (VEC && C::NPL > 1) {       // plane: cp / PIECES, at most 2
                const bool p1 = cp >= (unsigned)C::PIECES, p2 = C::NPL > 2 && cp >= 2u * C::PIECES;
                c = cp - (p2 ? 2u * C::PIECES : p1 ? (unsigned)C::PIECES : 0u);
                poff = p2 ? 2u * (unsigned)plane_bytes : p1 ? (unsigned)plane_bytes : 0u;
            }
            unsigned off = mad_u24(r, row_bytes, c * TB + poff);
            // lanes past the slab fill the room after it from the slab's
            // first piece
            if ((o + 1) * kThreads > P::NELEM && e >= (unsigned)P::NELEM) off = 0;
            if constexpr (VEC)
                lds_dma16_at(sbase, off, base + e0 * 16);
            else
                lds_dma4_at(sbase, off, base + e0 * 4);
        }
        return;
    }
    const unsigned long long in = (unsigned long long)g.in;
    const unsigned long long zsrc = (unsigned long long)zero_block + TB * lane;
#pragma unroll
    for (int o = 0; o < P::D; ++o) {
        const int e0 = (o * kWaves + wave) * 64;      // first transfer of the instruction
        const unsigned e = (unsigned)e0 + lane;
        const unsigned r = e / PER_ROW, cp = e - r * PER_ROW;
        const unsigned pl = VEC && C::NPL > 1 ? cp / C::PIECES : 0u;         // plane
        const unsigned c = VEC && C::NPL > 1 ? cp - pl * C::PIECES : cp;      // piece (or value)
        const int gy = wrap<BC>(sy0 + (int)r, g.ny);
        const int gx = wrap<BC>(sx0 + (int)(VEC ? c * C::CH : c), g.nx);
        bool ok = (o + 1) * kThreads <= P::NELEM || e < (unsigned)P::NELEM;
        if constexpr (BC == kBcZero) ok = ok && (unsigned)gy < (unsigned)g.ny && (unsigned)gx < (unsigned)g.nx;
        const unsigned long long at =
            in + (C::NPL > 1 ? pl * plane_bytes : 0ull) +
            ((unsigned long long)(unsigned)gy * (unsigned)g.nx + (unsigned)gx) * C::EB;
        const void *src = (const void *)(ok ? at : zsrc);
        if constexpr (VEC)
            lds_dma16(src, base + e0 * 16);
        else
            lds_dma4(src, base + e0 * 4);
    }
}

// The stored pair of staging row r whose first value is pair j's: two FP32
// values, or the word of two 16-bit values of each stored plane (assembled
// from the two words around it when the pair starts at an odd column).
template <int R1, int R2, int RAD, int STATE>
struct StagedPair {
    float x0, x1;
    unsigned w, wl, wm;    // hi (or binary16), lo and mid words
};

// The word of the two 16-bit values at staged value index col (col even, or
// odd and assembled from the two words around it).
template <bool ODD>
__device__ inline unsigned word16(const char *stage, int col) {
    if constexpr (!ODD) {
        return *reinterpret_cast<const unsigned *>(stage + 2 * col);
    } else {
        const unsigned *s = reinterpret_cast<const unsigned *>(stage + 2 * (col - 1));
        return __builtin_amdgcn_alignbyte(s[1], s[0], 2);
    }
}

template <int R1, int R2, int RAD, int STATE>
__device__ inline StagedPair<R1, R2, RAD, STATE> load_pair(const char *stage, int r, int j) {
    using C = ConvGeom<R1, R2, RAD, STATE>;
    const int col = r * C::NPL * C::SPITCH + C::P0 + 2 * j;
    StagedPair<R1, R2, RAD, STATE> v{0.f, 0.f, 0u, 0u, 0u};
    if constexpr (STATE == kStateF16) {
        v.w = word16<C::P0 % 2 != 0>(stage, col);
    } else if constexpr (STATE == kStatePlanes) {
        v.w = word16<C::P0 % 2 != 0>(stage, col);
        v.wl = word16<C::P0 % 2 != 0>(stage, col + C::SPITCH);
    } else if constexpr (STATE == kStatePlanes3) {
        v.w = word16<C::P0 % 2 != 0>(stage, col);
        v.wm = word16<C::P0 % 2 != 0>(stage, col + C::SPITCH);
        v.wl = word16<C::P0 % 2 != 0>(stage, col + 2 * C::SPITCH);
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
    } else if constexpr (STATE == kStatePlanes) {
        *reinterpret_cast<u2v *>(dst) = u2v{v.w, v.wl};
    } else if constexpr (STATE == kStatePlanes3) {
        unsigned *d = reinterpret_cast<unsigned *>(dst);
        d[0] = v.w;
        d[1] = v.wm;
        d[2] = v.wl;
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
// that would take too many registers (32 and more), two 16-bit dword indices
// per word (a converted slab is smaller than 256 KiB and its pairs are
// dword-aligned), unpacked at each use.  The packed word passes through an
// empty asm that takes a loop-varying value, so that the unpacked addresses
// are not hoisted out of the item loop and kept live (which would undo the
// packing).
template <int KC, int VPK>
struct GatherAddr {
    static constexpr bool PACK = KC * VPK >= 32;
    unsigned w[KC][PACK ? VPK / 2 : VPK];
    __device__ inline void set(int kc, int v, unsigned a) {
        if constexpr (PACK)
            w[kc][v >> 1] = (v & 1) ? (w[kc][v >> 1] | ((a >> 2) << 16)) : (a >> 2);
        else
            w[kc][v] = a;
    }
    __device__ inline unsigned get(int kc, int v, int salt) const {
        if constexpr (PACK) {
            unsigned x = w[kc][v >> 1];
            asm("" : "+v"(x) : "s"(salt));
            return (v & 1) ? ((x >> 14) & ~3u) : ((x & 0xffffu) << 2);
        } else {
            return w[kc][v];
        }
    }
};

// The band of a fused zero-halo launch (S radius-1 sweeps composed into one;
// paper Section 4.1 fuses three): the composed stencil applied to the
// zero-padded grid is exact only farther than S - 1 from the edges, and the
// products leave the points within that band (widened as BandBounds says)
// unwritten.  The band is cut into tiles -- its top and bottom rows in
// pieces kBand2W wide, its side columns (of the rows between) in pieces
// kBand2H tall -- and each tile is evaluated as S plain FP32 sweeps over
// LDS: the inputs within S of the tile, then the values of sweep s within
// S - s of it (zero outside the grid), then the tile's points.  Every value
// is summed in the fixed order (rows, then columns, fused multiply-adds).
constexpr int kBand2W = 256, kBand2H = 128;
// LDS floats: the input window and two levels of intermediate values
constexpr int kBand2Win = 2112, kBand2Lv = 1568, kBand2Lds = kBand2Win + 2 * kBand2Lv;
// (S <= 3: row tiles at most 2 rows deep, side tiles at most 5 columns wide)
static_assert(kBand2Win >= 8 * (kBand2W + 6) && kBand2Win >= (kBand2H + 6) * 11 &&
                  kBand2Lv >= 6 * (kBand2W + 4) && kBand2Lv >= (kBand2H + 4) * 9,
              "band tile windows");

struct Band2Tiles {
    int top, bot, L, R;          // band rows [0, top) and [bot, ny); columns [0, L) and [R, nx) between
    int cx, cy;                  // tiles per band row range, per side column range
    int n0, n1, n2, n3;          // top, bottom, left and right tiles
    __device__ inline Band2Tiles(const BandBounds &bb, int ny, int nx) {
        top = min(bb.b, ny);
        bot = max(ny - bb.b, top);
        L = min(bb.bl, nx);
        R = max(bb.br, L);
        cx = (nx + kBand2W - 1) / kBand2W;
        cy = (bot - top + kBand2H - 1) / kBand2H;
        n0 = top > 0 ? cx : 0;
        n1 = bot < ny ? cx : 0;
        n2 = L > 0 ? cy : 0;
        n3 = R < nx ? cy : 0;
    }
    __device__ inline int count() const { return n0 + n1 + n2 + n3; }
    // tile t: first row and column, rows and columns
    __device__ inline void box(int t, int ny, int nx, int *y0, int *x0, int *h, int *w) const {
        if (t < n0 + n1) {
            const bool f = t >= n0;
            const int c = f ? t - n0 : t;
            *y0 = f ? bot : 0;
            *h = f ? ny - bot : top;
            *x0 = c * kBand2W;
            *w = min(kBand2W, nx - *x0);
        } else {
            t -= n0 + n1;
            const bool f = t >= n2;
            const int c = f ? t - n2 : t;
            *y0 = top + c * kBand2H;
            *h = min(kBand2H, bot - *y0);
            *x0 = f ? R : 0;
            *w = f ? nx - R : L;
        }
    }
};

// Publish the workgroup's LDS writes: wait for this wave's LDS accesses
// (transfers to global memory left in flight), then barrier; the empty asm
// statements keep the compiler from moving LDS accesses across.
__device__ inline void band_publish() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One band tile (rows y0.., columns x0.., h x w points) after S sweeps.
// The input window is read from the grid into lds, or is already at lds +
// pre (pre >= 0: staged by LDS DMA, in the same layout).
template <int S>
__device__ inline void band_tile(const MmaJob &g, int y0, int x0, int h, int w, const float (&cw)[3][3],
                                 float *lds, int pre) {
    const float *in = static_cast<const float *>(g.in);
    float *out = static_cast<float *>(g.out);
    const float *src = lds + (pre >= 0 ? pre : 0);
    if (pre < 0) {
        const int W = w + 2 * S, n = (h + 2 * S) * W;
        for (int i = threadIdx.x; i < n; i += kThreads) {
            const int r = i / W, c = i - r * W;
            const int gy = y0 - S + r, gx = x0 - S + c;
            lds[i] = (gy >= 0 && gy < g.ny && gx >= 0 && gx < g.nx) ? in[(size_t)gy * g.nx + gx] : 0.f;
        }
        band_publish();
    }
#pragma unroll
    for (int st = 1; st <= S; ++st) {
        const int m = S - st;                  // sweep st's values reach m beyond the tile
        const int W = w + 2 * m, n = (h + 2 * m) * W, SW = W + 2;
        float *dst = lds + kBand2Win + ((st - 1) & 1) * kBand2Lv;
        for (int i = threadIdx.x; i < n; i += kThreads) {
            const int r = i / W, c = i - r * W;
            float acc = 0.f;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) acc = __builtin_fmaf(cw[dy][dx], src[(r + dy) * SW + c + dx], acc);
            const int gy = y0 - m + r, gx = x0 - m + c;
            if (st < S)
                dst[i] = (gy >= 0 && gy < g.ny && gx >= 0 && gx < g.nx) ? acc : 0.f;
            else
                out[(size_t)gy * g.nx + gx] = acc;
        }
        band_publish();                        // (the last one: the next tile reuses the LDS)
        src = dst;
    }
}

// The first of the band tiles wg, wg + nb, ... (numbered over the grids of
// the launch in order): its grid and number, or false if there is none.
__device__ inline bool first_band_tile(const MmaArgs &p, int wg, int nb, int *jj, int *tt) {
    int base = 0;
    for (int j = 0; j < p.njobs; ++j) {
        const MmaJob &g = p.job[j];
        const int n = Band2Tiles(band_bounds(p, g), g.ny, g.nx).count();
        const int t = base <= wg ? wg - base : (nb - (base - wg) % nb) % nb;
        if (t < n) {
            *jj = j;
            *tt = t;
            return true;
        }
        base += n;
    }
    return false;
}

// LDS DMA of a band tile's input window (rows y0 - S.., columns x0 - S..,
// row-major, zero outside the grid) into a staging slab: the same count of
// transfers per wave as an item's (4-byte ones: the window's rows start
// anywhere), so that the pipeline's waits count it as one.
template <int R1, int R2, int RAD, int STATE, bool VEC>
__device__ inline void issue_band_window(const void *zero_block, const MmaJob &g, char *stage, int y0, int x0,
                                         int h, int w, int S) {
    using C = ConvGeom<R1, R2, RAD, STATE>;
    using P = CPipe<R1, R2, RAD, STATE, VEC>;
    static_assert(P::D * kThreads >= kBand2Win && P::D * kThreads * 4 <= C::STAGE_ALLOC, "band window transfers");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned base = lds_addr_of(stage);
    const int W = w + 2 * S, n = (h + 2 * S) * W;
    const float *in = static_cast<const float *>(g.in);
    const float *zf = static_cast<const float *>(zero_block);
#pragma unroll
    for (int o = 0; o < P::D; ++o) {
        const int e0 = (o * kWaves + wave) * 64;
        const int e = e0 + lane;
        const int r = e / W, c = e - r * W;
        const int gy = y0 - S + r, gx = x0 - S + c;
        const bool ok = e < n && gy >= 0 && gy < g.ny && gx >= 0 && gx < g.nx;
        lds_dma4(ok ? static_cast<const void *>(in + (size_t)gy * g.nx + gx) : static_cast<const void *>(zf + lane),
                 base + e0 * 4);
    }
}

// Workgroup wg of nb computes, after its work items (its LDS free), the
// band tiles wg, wg + nb, ... of all grids of the launch (numbered over
// the grids in order); the first one's window may already be staged at
// lds + pre (pre >= 0).
__device__ inline void band_share(const MmaArgs &p, int wg, int nb, float *lds, int pre) {
    if (p.edge_steps < 2) return;
    float w[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) w[i][c] = p.edge_w32[i * 3 + c];
    int base = 0;
    for (int j = 0; j < p.njobs; ++j) {
        const MmaJob &g = p.job[j];
        const Band2Tiles bt(band_bounds(p, g), g.ny, g.nx);
        const int n = bt.count();
        for (int t = base <= wg ? wg - base : (nb - (base - wg) % nb) % nb; t < n; t += nb) {
            int y0, x0, h, tw;
            bt.box(t, g.ny, g.nx, &y0, &x0, &h, &tw);
            if (p.edge_steps == 3)
                band_tile<3>(g, y0, x0, h, tw, w, lds, pre);
            else
                band_tile<2>(g, y0, x0, h, tw, w, lds, pre);
            pre = -1;
        }
        base += n;
    }
}

// Multiply one work item out of the converted slab and write its outputs.
// Wave w owns units (w / NCOLS) * U + u of unit column w % NCOLS; gaddr holds
// the lane's gather addresses (bytes from the slab) for unit 0.
template <int R1, int R2, int KC, int RAD, int MODE, int PART, int STATE, bool VEC>
__device__ inline void compute_conv(float inv_sigma, const MmaJob &g, const char *conv,
                                    const uint4 (&ahi)[R1 * R2 / 16][KC], const uint4 (&alo)[R1 * R2 / 16][KC],
                                    const uint4 (&amid)[R1 * R2 / 16][KC], const unsigned (&aidx)[R1 * R2 / 16][KC],
                                    const GatherAddr<KC, (MODE == kSparse) ? 8 : 4> &gaddr, int X0, int Y0,
                                    int salt, const BandBounds &bb) {
    using C = ConvGeom<R1, R2, RAD, STATE>;
    using G = typename C::G;
    constexpr int MB = G::MB;
    constexpr int VPK = (MODE == kSparse) ? 8 : 4;
    constexpr bool SPLIT = STATE != kStateF16;      // hi and lo B operands
    constexpr bool THREE = STATE == kStatePlanes3;  // and mid operands
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
        // three-part products keep hi*hi, hi*mid + mid*hi, and hi*lo +
        // lo*hi + mid*mid, each in accumulators of their own
        f4 accm[MB], acc1[MB], acc2[MB], acc3[MB], acc4[MB], acc5[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            accm[mb] = f4{0.f, 0.f, 0.f, 0.f};
            acc1[mb] = f4{0.f, 0.f, 0.f, 0.f};
            acc2[mb] = f4{0.f, 0.f, 0.f, 0.f};
            acc3[mb] = f4{0.f, 0.f, 0.f, 0.f};
            acc4[mb] = f4{0.f, 0.f, 0.f, 0.f};
            acc5[mb] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            unsigned bh[VPK], bl[VPK], bm[VPK];
#pragma unroll
            for (int v = 0; v < VPK; ++v) {
                const char *a = conv + gaddr.get(kc, v, salt + u) + uoff;
                if constexpr (THREE) {
                    const unsigned *w = reinterpret_cast<const unsigned *>(a);
                    bh[v] = w[0];
                    bm[v] = w[1];
                    bl[v] = w[2];
                } else if constexpr (SPLIT) {
                    const u2v w = *reinterpret_cast<const u2v *>(a);
                    bh[v] = w.x;
                    bl[v] = w.y;
                    bm[v] = 0;
                } else {
                    bh[v] = *reinterpret_cast<const unsigned *>(a);
                    bl[v] = 0;
                    bm[v] = 0;
                }
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) accm[mb] = mma<MODE, PART>(ahi[mb][kc], bh, accm[mb], aidx[mb][kc]);
            if constexpr (THREE) {
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    acc1[mb] = mma<MODE, PART>(ahi[mb][kc], bm, acc1[mb], aidx[mb][kc]);
                    acc2[mb] = mma<MODE, PART>(amid[mb][kc], bh, acc2[mb], aidx[mb][kc]);
                    acc3[mb] = mma<MODE, PART>(ahi[mb][kc], bl, acc3[mb], aidx[mb][kc]);
                    acc4[mb] = mma<MODE, PART>(alo[mb][kc], bh, acc4[mb], aidx[mb][kc]);
                    acc5[mb] = mma<MODE, PART>(amid[mb][kc], bm, acc5[mb], aidx[mb][kc]);
                }
            } else if constexpr (SPLIT) {
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
            // the band of a fused zero-halo launch is written by band_item
            const int gya = Y0 + gyr;
            const bool row_ok = gyr < rows_left && gya >= bb.b && gya < g.ny - bb.b;
            float ys[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if constexpr (!SPLIT)
                    ys[i] = accm[mb][i];
                else if constexpr (THREE)
                    ys[i] = accm[mb][i] + ((acc1[mb][i] + acc2[mb][i]) + ((acc3[mb][i] + acc4[mb][i]) + acc5[mb][i]));
                else if constexpr (MERGE)
                    ys[i] = accm[mb][i] + acc1[mb][i] * inv_sigma;
                else
                    ys[i] = accm[mb][i] + (acc1[mb][i] + acc2[mb][i]) * inv_sigma;
            }
            if constexpr (STATE == kStatePlanes3) {
                // bfloat16 hi = RNE(y), mid = RNE(y - hi), lo = RNE(y - hi -
                // mid) (exact differences: together they hold y); rows are
                // a multiple of 8 values, so the four outputs are all in or
                // all out
                unsigned short h[3][4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float r = ys[i];
#pragma unroll
                    for (int t = 0; t < 3; ++t) {
                        const __bf16 pb = (__bf16)r;
                        h[t][i] = __builtin_bit_cast(unsigned short, pb);
                        r -= (float)pb;
                    }
                }
                unsigned short *out = static_cast<unsigned short *>(g.out);
                const size_t plane = (size_t)g.ny * g.nx;
                const unsigned o2 = row_ok && gx < g.nx ? (unsigned)(gyr * g.nx + gx) * 2u : kOob;
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const u2v hv = {(unsigned)h[t][0] | ((unsigned)h[t][1] << 16),
                                    (unsigned)h[t][2] | ((unsigned)h[t][3] << 16)};
                    const __amdgpu_buffer_rsrc_t rs =
                        uniform_rsrc(out + t * plane + (size_t)Y0 * g.nx, rows_left * g.nx * 2);
                    __builtin_amdgcn_raw_buffer_store_b64(hv, rs, o2, 0, 0);
                }
            } else if constexpr (STATE == kStatePlanes) {
                // bfloat16 hi = RNE(y), lo = RNE(y - hi); rows are a
                // multiple of 8 values, so the four outputs are all in or
                // all out
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
            } else if constexpr (STATE == kStateF16) {
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
                    const unsigned o4 =
                        row_ok && gx < g.nx && gx >= bb.bl && gx < bb.br ? (unsigned)(gyr * g.nx + gx) * 4u : kOob;
                    __builtin_amdgcn_raw_buffer_store_b128(yv, orsrc, o4, 0, 0);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const unsigned o1 = row_ok && gx + i < g.nx && gx + i >= bb.bl && gx + i < bb.br
                                                ? (unsigned)(gyr * g.nx + gx + i) * 4u
                                                : kOob;
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
    static_assert(STATE != kStateF32 || C::CONV_BYTES >= 4 * kBand2Lds, "band tiles need more LDS");
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
    if (first >= total) {
        if constexpr (STATE == kStateF32) band_share(p, blockIdx.x, nwg, reinterpret_cast<float *>(lds), -1);
        return;
    }

    // gather addresses of unit 0: the tile's patch origin in the converted
    // slab plus the plan's offset of each B register
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4;
    GatherAddr<KC, VPK> gaddr;
    static_assert(!GatherAddr<KC, VPK>::PACK || C::CONV_BYTES <= 4 * 65536, "16-bit gather dword indices");
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
    uint4 ahi[MB][KC], alo[MB][KC], amid[MB][KC];
    unsigned aidx[MB][KC];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const int t = (mb * KC + kc) * 64 + lane;
            ahi[mb][kc] = p.a_hi[t];
            alo[mb][kc] = STATE != kStateF16 ? p.a_lo[t] : uint4{0u, 0u, 0u, 0u};
            amid[mb][kc] = STATE == kStatePlanes3 ? p.a_mid[t] : uint4{0u, 0u, 0u, 0u};
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
    // the first transfer round past this workgroup's last item stages the
    // window of its first band tile instead (fused zero-halo launches), so
    // that the band pass after the items starts with its inputs in LDS
    // (round n_items: the first past the last item)
    const int n_items = (total - first + stride - 1) / stride;
    int band_j = -1, band_t = 0;
    if constexpr (STATE == kStateF32)
        if (p.edge_steps < 2 || !first_band_tile(p, blockIdx.x, nwg, &band_j, &band_t)) band_j = -1;
    auto issue = [&](int s) {
        if constexpr (STATE == kStateF32) {
            if (band_j >= 0 && s == n_items) {
                const MmaJob g = p.job[band_j];
                int y0, x0, h, tw;
                Band2Tiles(band_bounds(p, g), g.ny, g.nx).box(band_t, g.ny, g.nx, &y0, &x0, &h, &tw);
                issue_band_window<R1, R2, RAD, STATE, VEC>(p.zeros, g, stage(s % NS), y0, x0, h, tw,
                                                           p.edge_steps);
                return;
            }
        }
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
        const BandBounds bb = STATE == kStateF32 ? band_bounds(p, g) : BandBounds{0, 0, g.nx};
        compute_conv<R1, R2, KC, RAD, MODE, PART, STATE, VEC>(inv_sigma, g, conv, ahi, alo, amid, aidx, gaddr, X0, Y0,
                                                              s * G::U, bb);
        if (first + (s + 1) * stride >= total) break;
    }
    // the pipeline always runs NS items ahead: let those transfers land
    // before the workgroup's LDS is released
    wait_vmcnt<0>();
    if constexpr (STATE == kStateF32) {
        __builtin_amdgcn_s_barrier();            // every wave is done with the slabs
        band_share(p, blockIdx.x, nwg, reinterpret_cast<float *>(lds),
                   band_j >= 0 ? (C::CONV_BYTES + (n_items % NS) * C::STAGE_ALLOC) / 4 : -1);
    }
}

template <int R1, int R2, int KC, int RAD, int MODE, int PART, int STATE, bool VEC, int BC>
static hipError_t launch_c_bc(const MmaArgs &a, hipStream_t s) {
    int cus = 0, xcds = 0;
    if (const hipError_t e = device_shape(&cus, &xcds); e != hipSuccess) return e;
    MmaArgs b = a;
    b.nxcd = xcds;
    const int wgs = a.total_items < cus ? a.total_items : cus;
    hipLaunchKernelGGL((k_mma2c<R1, R2, KC, RAD, MODE, PART, STATE, VEC, BC>), dim3(wgs), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

// Number the jobs' work items, then pick the variant every job of the launch
// can use: 16-byte pieces or 4-byte values (FP32 rows that are not a multiple
// of 4 values), and the cheapest boundary handling valid for all of them.
// Binary16 and planes rows must be a multiple of 8 values (the planner
// checks).
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
    if constexpr (STATE != kStateF32) {
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
