// 3-D stencil sweep as a structured-sparse (or dense) matrix product on
// gfx950 matrix cores, FP32 state split into hi + lo parts once per plane.
//
// The 3-D staircase matrix A' has one block level more than in 2-D: a patch
// is 2r+1 z planes of the 2-D patch, and each output tile of r2 x r1 points
// in one z plane uses all of them.  The matching runs per plane (the planes'
// columns never share a 4-group here), and every plane's K columns are
// padded to whole MMA chunks, so that a chunk gathers from a single input
// plane.  A work item is a 256 x WGH column of the grid over ZC planes; the
// workgroup streams the input planes through a ring of LDS slabs filled by
// LDS DMA several planes ahead.  Each input plane, once landed, is converted
// into hi and lo word pairs (the 2-D kernels' bank-spread converted layout),
// gathered into B registers once and multiplied by the A blocks of all 2r+1
// plane offsets, accumulating into the 2r+1 output planes it contributes
// to; the oldest of those is complete after the plane and is stored.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mma2d_impl.hpp"

namespace ss {

template <int R1, int R2, int RAD, bool VEC, int NPR = Mma3Geom<R1, R2, RAD>::NP>
struct Pipe3 {
    using G = Mma3Geom<R1, R2, RAD>;
    static constexpr int DRW = (G::SROWS + kWaves - 1) / kWaves;   // rows each wave loads per plane
    // a row is 264 values from HL-4: 64 lanes x 16 bytes and 2 lanes x 16
    // bytes, or 4 x 64 lanes x 4 bytes and 8 lanes x 4 bytes
    static constexpr int DMA_PER_ROW = VEC ? 2 : 5;
    static constexpr int D = DRW * DMA_PER_ROW;                    // VMEM loads per wave per plane
    // VMEM stores per wave per output plane: one 16-byte store per M block,
    // or four 4-byte ones (rows not 16-byte aligned)
    static constexpr int M = G::MB * (VEC ? 1 : 4);
    static constexpr int A = 2 * RAD;                              // steps before the first store
    // Step l waits for plane l + 1 (its B operands are gathered while the
    // matrix cores multiply plane l).  VMEM operations a wave has issued
    // after the loads of plane l + 1 at that point: the loads of the NP-3
    // planes issued after it and at most the stores of the NP-2 steps since.
    // From step A + NP - 2 on that is exact (WS); before it fewer stores
    // follow, and waiting for WL (no stores) waits for a few more loads than
    // needed.  Plane 0 is waited for before the first step (W0).
    static constexpr int W0 = (NPR - 2) * D;
    static constexpr int WL = (NPR - 3) * D;
    static constexpr int WS = (NPR - 3) * D + (NPR - 2) * M;
    static constexpr int STEADY = A + NPR - 2;
};

// Issue the transfers of input plane z (already wrapped; outside the grid
// with a zero halo) into a ring slot.  Values outside a zero-halo grid come
// from the 1 KiB zero block, each lane from its own part of it.  Every wave moves the slab rows wave,
// wave + 8, ... (clamped to the last row, so that all waves issue the same
// count); rows are item constants, passed as element offsets (-1: outside
// the grid) with the slab row addresses.
template <int R1, int R2, int RAD, bool VEC, int BC>
__device__ inline void issue_plane(const MmaJob &g, const float *zf, unsigned slot_lds,
                                   const int (&row_off)[Pipe3<R1, R2, RAD, VEC>::DRW],
                                   const unsigned (&row_lds)[Pipe3<R1, R2, RAD, VEC>::DRW], int X0, int z) {
    using P = Pipe3<R1, R2, RAD, VEC>;
    const int lane = threadIdx.x & 63;
    const bool z_ok = BC != kBcZero || (z >= 0 && z < g.nz);
    const float *in = static_cast<const float *>(g.in) + (size_t)(z_ok ? z : 0) * g.ny * g.nx;
    if constexpr (VEC) {
        // chunk c of the row holds columns X0 - 4 + 4c (c = 0..65)
        const int gxa = wrap<BC>(X0 - 4 + 4 * lane, g.nx);
        const int gxb = wrap<BC>(X0 + 252 + 4 * lane, g.nx);
        const bool oka = BC != kBcZero || (gxa >= 0 && gxa < g.nx);
        const bool okb = BC != kBcZero || (gxb >= 0 && gxb < g.nx);
#pragma unroll
        for (int d = 0; d < P::DRW; ++d) {
            const bool row_ok = z_ok && row_off[d] >= 0;
            const float *row = in + row_off[d];
            lds_dma16(row_ok && oka ? row + gxa : zf + 4 * lane, slot_lds + row_lds[d]);
            if (lane < 2) lds_dma16(row_ok && okb ? row + gxb : zf + 4 * lane, slot_lds + row_lds[d] + 1024);
        }
    } else {
#pragma unroll
        for (int d = 0; d < P::DRW; ++d) {
            const bool row_ok = z_ok && row_off[d] >= 0;
            const float *row = in + row_off[d];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int gx = wrap<BC>(X0 - 4 + 64 * h + lane, g.nx);
                const bool ok = BC != kBcZero || (gx >= 0 && gx < g.nx);
                lds_dma4(row_ok && ok ? row + gx : zf + lane, slot_lds + row_lds[d] + 256 * h);
            }
            if (lane < 8) {
                const int gx = wrap<BC>(X0 + 252 + lane, g.nx);
                const bool ok = BC != kBcZero || (gx >= 0 && gx < g.nx);
                lds_dma4(row_ok && ok ? row + gx : zf + lane, slot_lds + row_lds[d] + 1024);
            }
        }
    }
}

// Gather offset of B register v with the word passed through an empty asm
// that takes the plane index: the unpacking stays inside the plane loop (it
// is not hoisted and kept live), and since the asm touches no memory the LDS
// reads of a plane can be issued together.
template <int VPK>
__device__ inline int plane_off(const unsigned (&o2)[VPK / 2], int v, int l) {
    unsigned w = o2[v >> 1];
    asm("" : "+v"(w) : "s"(l));
    return (v & 1) ? (int)(w >> 16) : (int)(w & 0xffffu);
}

// Publish the workgroup's LDS writes to all its waves: wait for this
// wave's (lgkmcnt(0), VMEM transfers left in flight), then barrier; the
// empty asm statements keep the compiler from moving LDS accesses across.
__device__ inline void lds_publish() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// The band of a fused zero-halo launch of two radius-1 sweeps (composed
// into one radius-2 stencil): applied to the zero-padded grid, the composed
// stencil is exact only at points at least one away from every face (paper
// Section 4.1 fuses sweeps; recomputing the band keeps the zero-halo result
// exact).  Along x the band is widened to kBandX0 = 4 columns a side, the
// work items' 16-byte store granularity, so that no item store straddles
// it.  It is cut into boxes: the first and last planes in 32 x 64 (rows x
// columns) tiles; the first and last rows of the planes between in 32 x 64
// (planes x columns) tiles; the first and last four columns of the rows
// between in 32 x 32 x 4 (planes x rows x columns) boxes.
constexpr int kBandT = 32, kBandW = 64, kBandX0 = 4;
// LDS of a box's windows (floats) and window values a thread loads
constexpr int kBandWin = 12288, kBandMid = 7168, kBandRegs = 24;

struct BandBox {
    int z0, y0, x0, ez, ey, ex;
    int kind;                    // 0: plane tile, 1: row tile, 2: column box
};

struct BandTiles3 {
    int mz, my;                  // planes and rows strictly inside
    int fz, fy, fx;              // faces of each kind: 1, or 2 if the grid is wide enough
    int tz, ty, tx;              // tiles per face of each kind
    int xl, xr;                  // column boxes: [0, xl) and [xr, nx)
    __device__ inline BandTiles3(int nz, int ny, int nx) {
        mz = max(nz - 2, 0);
        my = max(ny - 2, 0);
        fz = min(nz, 2);
        fy = min(ny, 2);
        xl = min(kBandX0, nx);
        xr = max(xl, nx - kBandX0);
        fx = xr < nx ? 2 : 1;
        const int cx = (nx + kBandW - 1) / kBandW, czm = (mz + kBandT - 1) / kBandT;
        tz = (ny + kBandT - 1) / kBandT * cx;
        ty = czm * cx;
        tx = czm * ((my + kBandT - 1) / kBandT);
    }
    __device__ inline int count() const { return fz * tz + fy * ty + fx * tx; }
    __device__ inline BandBox box(int t, int nz, int ny, int nx) const {
        const int cx = (nx + kBandW - 1) / kBandW;
        if (t < fz * tz) {
            const int f = t / tz, r = t % tz;
            const int y0 = (r / cx) * kBandT, x0 = (r % cx) * kBandW;
            return BandBox{f ? nz - 1 : 0, y0, x0, 1, min(kBandT, ny - y0), min(kBandW, nx - x0), 0};
        }
        t -= fz * tz;
        if (t < fy * ty) {
            const int f = t / ty, r = t % ty;
            const int z0 = 1 + (r / cx) * kBandT, x0 = (r % cx) * kBandW;
            return BandBox{z0, f ? ny - 1 : 0, x0, min(kBandT, mz + 1 - z0), 1, min(kBandW, nx - x0), 1};
        }
        t -= fy * ty;
        const int f = t / tx, r = t % tx, cy = (my + kBandT - 1) / kBandT;
        const int z0 = 1 + (r / cy) * kBandT, y0 = 1 + (r % cy) * kBandT;
        return BandBox{z0, y0, f ? xr : 0, min(kBandT, mz + 1 - z0), min(kBandT, my + 1 - y0), f ? nx - xr : xl, 2};
    }
};

// Exact two-sweep values of band boxes of at most EZ x EY x EX points
// (FP32, fixed order): the inputs within two of a box (zero outside the
// grid) are loaded into registers (band_load, one box ahead of the
// arithmetic), then put into LDS; the first-sweep values within one of the
// box (zero outside the grid) go to LDS; then the second sweep at the box's
// points (band_compute).  Window shapes are compile-time, so index
// arithmetic is by constants.
template <int EZ, int EY, int EX>
struct BandWin {
    static constexpr int WZ = EZ + 4, WY = EY + 4, WX = EX + 4, NW = WZ * WY * WX;
    static constexpr int MY = EY + 2, MX = EX + 2, NM = (EZ + 2) * MY * MX;
    static constexpr int NO = EZ * EY * EX;
    static constexpr int NR = (NW + kThreads - 1) / kThreads;     // window values per thread
    static_assert(NW <= kBandWin && NM <= kBandMid && NR <= kBandRegs, "band windows");
};

template <int EZ, int EY, int EX>
__device__ inline void band_load(const MmaJob &g, const BandBox &bx, float (&v)[kBandRegs]) {
    using B = BandWin<EZ, EY, EX>;
    const float *in = static_cast<const float *>(g.in);
#pragma unroll
    for (int r = 0; r < B::NR; ++r) {
        const int i = threadIdx.x + r * kThreads;
        const int k = i % B::WX, j = (i / B::WX) % B::WY, l = i / (B::WX * B::WY);
        const int z = bx.z0 - 2 + l, y = bx.y0 - 2 + j, x = bx.x0 - 2 + k;
        const bool ok = i < B::NW && z >= 0 && z < g.nz && y >= 0 && y < g.ny && x >= 0 && x < g.nx;
        v[r] = ok ? in[((size_t)z * g.ny + y) * g.nx + x] : 0.f;
    }
}

template <int EZ, int EY, int EX>
__device__ inline void band_compute(const MmaJob &g, const BandBox &bx, const float (&v)[kBandRegs], const float (&w)[27],
                                    float *lds) {
    using B = BandWin<EZ, EY, EX>;
    float *win = lds, *mid = lds + kBandWin;
#pragma unroll
    for (int r = 0; r < B::NR; ++r)
        if (threadIdx.x + r * kThreads < B::NW) win[threadIdx.x + r * kThreads] = v[r];
    lds_publish();
    // first-sweep values: threads take them with the window's thin axis
    // slowest, so that a wave's values outside the grid (a whole layer of
    // the thin axis) are skipped together
    constexpr int MZ = EZ + 2;
#pragma unroll 1
    for (int r = 0; r < (B::NM + kThreads - 1) / kThreads; ++r) {
        const int i = threadIdx.x + r * kThreads;
        if (i < B::NM) {
            int l, j, k;
            if constexpr (EX == 1) {
                k = i / (MZ * B::MY);
                j = i % B::MY;
                l = (i / B::MY) % MZ;
            } else {
                k = i % B::MX;
                j = (i / B::MX) % B::MY;
                l = i / (B::MX * B::MY);
            }
            const int z = bx.z0 - 1 + l, y = bx.y0 - 1 + j, x = bx.x0 - 1 + k;
            const bool ok = z >= 0 && z < g.nz && y >= 0 && y < g.ny && x >= 0 && x < g.nx;
            float m = 0.f;
            if (ok) {
#pragma unroll
                for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 3; ++dx)
                            m = __builtin_fmaf(w[(dz * 3 + dy) * 3 + dx],
                                               win[((l + dz) * B::WY + j + dy) * B::WX + k + dx], m);
            }
            mid[(l * B::MY + j) * B::MX + k] = m;
        }
    }
    lds_publish();
#pragma unroll 1
    for (int r = 0; r < (B::NO + kThreads - 1) / kThreads; ++r) {
        const int i = threadIdx.x + r * kThreads;
        const int k = i % EX, j = (i / EX) % EY, l = i / (EX * EY);
        if (i < B::NO && l < bx.ez && j < bx.ey && k < bx.ex) {
            float acc = 0.f;
#pragma unroll
            for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx)
                        acc = __builtin_fmaf(w[(dz * 3 + dy) * 3 + dx],
                                             mid[((l + dz) * B::MY + j + dy) * B::MX + k + dx], acc);
            static_cast<float *>(g.out)[((size_t)(bx.z0 + l) * g.ny + bx.y0 + j) * g.nx + bx.x0 + k] = acc;
        }
    }
    // the next box reuses the windows
    lds_publish();
}

// This workgroup's boxes of one kind (tiles first, first + nb, ... below
// end, numbered within the grid), the loads of each box issued before the
// arithmetic of the one before.
template <int EZ, int EY, int EX>
__device__ inline void band_kind(const MmaJob &g, const BandTiles3 &bt, int first, int end, int nb,
                                 const float (&w)[27], float *lds) {
    if (first >= end) return;
    float v[kBandRegs], nv[kBandRegs];
    BandBox bx = bt.box(first, g.nz, g.ny, g.nx);
    band_load<EZ, EY, EX>(g, bx, v);
    for (int t = first; t < end; t += nb) {
        const BandBox cur = bx;
        if (t + nb < end) {
            bx = bt.box(t + nb, g.nz, g.ny, g.nx);
            band_load<EZ, EY, EX>(g, bx, nv);
        }
        band_compute<EZ, EY, EX>(g, cur, v, w, lds);
#pragma unroll
        for (int r = 0; r < kBandRegs; ++r) v[r] = nv[r];
    }
}

// Workgroup wg of nb computes, after its work items (its LDS free), the
// band boxes wg, wg + nb, ... of all grids of a fused zero-halo launch
// (numbered over the grids in order).
__device__ inline void band_share3(const MmaArgs &p, int wg, int nb, float *lds) {
    if (p.edge_steps < 2) return;
    float w[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) w[i] = p.edge_w32[i];
    int base = 0;
    for (int j = 0; j < p.njobs; ++j) {
        const MmaJob &g = p.job[j];
        const BandTiles3 bt(g.nz, g.ny, g.nx);
        // this workgroup's first box of the grid, then the kinds' ranges
        const int first = base <= wg ? wg - base : (nb - (base - wg) % nb) % nb;
        const int e0 = bt.fz * bt.tz, e1 = e0 + bt.fy * bt.ty, e2 = bt.count();
        const int f1 = first >= e0 ? first : first + (e0 - first + nb - 1) / nb * nb;
        const int f2 = f1 >= e1 ? f1 : f1 + (e1 - f1 + nb - 1) / nb * nb;
        band_kind<1, kBandT, kBandW>(g, bt, first, e0, nb, w, lds);
        band_kind<kBandT, 1, kBandW>(g, bt, f1, e1, nb, w, lds);
        band_kind<kBandT, kBandT, kBandX0>(g, bt, f2, e2, nb, w, lds);
        base += e2;
    }
}

// Calls f(integral_constant<R>, l0 + R) for R = 0..N-1 while l0 + R < n.
template <int R, int N, typename F>
__device__ inline void unroll_steps(F &f, int l0, int n) {
    if constexpr (R < N) {
        if (l0 + R < n) {
            f(std::integral_constant<int, R>{}, l0 + R);
            unroll_steps<R + 1, N>(f, l0, n);
        }
    }
}

// BAND: a fused zero-halo launch; the items leave the band (Band3) unwritten
// and every workgroup computes a share of it after its items.
template <int R1, int R2, int KC, int RAD, int MODE, int PART, bool VEC, int BC, bool BAND>
__global__ __launch_bounds__(kThreads, 1) void k_mma3d(MmaArgs p) {
    using G = Mma3Geom<R1, R2, RAD>;
    using C = Conv3Geom<R1, R2, RAD>;
    constexpr int NP = C::NP;
    using P = Pipe3<R1, R2, RAD, VEC, NP>;
    constexpr int MB = G::MB;
    constexpr int VPK = (MODE == kSparse) ? 8 : 4;
    constexpr int NZ = 2 * RAD + 1;          // plane offsets of the stencil
    constexpr int CPP = KC / NZ;             // K chunks per input plane
    static_assert(CPP * NZ == KC, "chunks must not straddle planes");
    // the converted plane, then the ring of staged planes
    __shared__ __attribute__((aligned(16))) char lds[C::CONV_BYTES + NP * G::PLANE_BYTES];
    char *conv = lds;
    char *ring = lds + C::CONV_BYTES;
    const unsigned lds0 = lds_addr_of(ring);

    const float sigma = 1.0f / p.inv_sigma;
    const float inv_sigma = p.inv_sigma;
    const float *zf = static_cast<const float *>(p.zeros);
    const int bnd = BAND ? p.edge_rad * (p.edge_steps - 1) : 0;
    // XCD-aware contiguous item ranges, as in the 2-D kernel
    const int nxcd = p.nxcd;
    const int nwg = gridDim.x;
    const int xcd = blockIdx.x % nxcd;
    const int stride = nwg / nxcd + (xcd < nwg % nxcd ? 1 : 0);
    const int before = xcd * (nwg / nxcd) + min(xcd, nwg % nxcd);
    const int range_begin = (int)((long long)p.total_items * before / nwg);
    const int range_end = (int)((long long)p.total_items * (before + stride) / nwg);
    const int first = range_begin + blockIdx.x / nxcd;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q = lane >> 4;
    // every plane has the same K order (shifted by whole planes), so the
    // gather offsets of its CPP chunks serve all plane offsets
    unsigned off2[CPP][VPK / 2];
#pragma unroll
    for (int c = 0; c < CPP; ++c)
#pragma unroll
        for (int v = 0; v < VPK; v += 2)
            off2[c][v / 2] = (unsigned)p.boff[(c * 4 + q) * VPK + v] |
                             ((unsigned)p.boff[(c * 4 + q) * VPK + v + 1] << 16);
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
    wait_vmcnt<0>();

    const int n = lane & 15;
    const int tx_t = n % G::NBX, ty_t = n / G::NBX;
    const int nbc = wave % kNbCols, nb = wave / kNbCols;
    const int srow0 = nb * G::NBH + ty_t * R2;  // tile's first output row in the item
    // slab rows this wave moves (LDS byte offset within a slot)
    unsigned row_lds[P::DRW];
#pragma unroll
    for (int d = 0; d < P::DRW; ++d) row_lds[d] = min(wave + d * kWaves, G::SROWS - 1) * G::CPITCH * 4;
    // byte offset of the tile's patch origin within the converted plane
    const int tbo = (srow0 * C::ROWC + C::pos((nbc * 128 + tx_t * R1) / 2)) * 4;

#pragma unroll 1
    for (int it = first; it < range_end; it += stride) {
        // item -> job, band, row block, z chunk
        int j = 0;
        for (int t = 1; t < p.njobs; ++t) j += it >= p.job[t].item0 ? 1 : 0;
        // a copy in registers: the transfers' memory clobbers would
        // otherwise make every use reload the job from the argument block
        const MmaJob g = p.job[j];
        const int nbands = (g.nx + kBandX - 1) / kBandX, nrb = (g.ny + G::WGH - 1) / G::WGH;
        int local = it - g.item0;
        const int X0 = __builtin_amdgcn_readfirstlane((local % nbands) * kBandX);
        local /= nbands;
        const int Y0 = __builtin_amdgcn_readfirstlane((local % nrb) * G::WGH);
        const int z0 = __builtin_amdgcn_readfirstlane((local / nrb) * g.zc);
        const int nzc = min(g.zc, g.nz - z0);
        const int nload = nzc + 2 * RAD;   // input planes z0-RAD .. z0+nzc-1+RAD
        // element offsets of this wave's slab rows within a plane (-1 outside)
        int row_off[P::DRW];
#pragma unroll
        for (int d = 0; d < P::DRW; ++d) {
            const int gy = wrap<BC>(Y0 - RAD + min(wave + d * kWaves, G::SROWS - 1), g.ny);
            row_off[d] = (BC != kBcZero || (gy >= 0 && gy < g.ny)) ? gy * g.nx : -1;
        }
        auto issue = [&](int l) {
            const int zz = wrap<BC>(z0 - RAD + min(l, nload - 1), g.nz);
            issue_plane<R1, R2, RAD, VEC, BC>(g, zf, lds0 + (l % NP) * G::PLANE_BYTES, row_off, row_lds, X0, zz);
        };
#pragma unroll 1
        for (int l = 0; l < NP - 1; ++l) issue(l);
        const int rows_left = min(G::WGH, g.ny - Y0);
        const int xbase = X0 + nbc * 128 + tx_t * R1;
        // output plane z0 + l - 2*RAD + i accumulates at step l in slot
        // (i + l) % NZ; hi*hi in accm, hi*lo and lo*hi together in acc1
        // (issued a whole pass over the plane offsets apart, so that no
        // product waits for the one before it)
        f4 accm[NZ][MB], acc1[NZ][MB];
#pragma unroll
        for (int i = 0; i < NZ; ++i)
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                accm[i][mb] = f4{0.f, 0.f, 0.f, 0.f};
                acc1[i][mb] = f4{0.f, 0.f, 0.f, 0.f};
            }
        // B operands of two planes, the one multiplied and the next one
        // (one plane in the dense 4-byte-row variants, which gather after
        // the products for want of registers)
        constexpr int NB = (VEC || MODE == kSparse) ? 2 : 1;
        unsigned bh[NB][CPP][VPK], bl[NB][CPP][VPK];
        // staged plane l -> the converted plane: every pair split once into
        // its hi and lo words (all reads of a thread first, then its writes)
        auto convert = [&](int l) {
            constexpr int NPR = G::SROWS * C::NPAIR;
            constexpr int PER = (NPR + kThreads - 1) / kThreads;
            // pairs read before they are split and written (one at a time in the
            // 4-byte-row variants, whose stores take more registers)
            constexpr int BATCH = VEC ? 3 : 1;
            const float *st = reinterpret_cast<const float *>(ring + (l % NP) * G::PLANE_BYTES);
#pragma unroll
            for (int r0 = 0; r0 < PER; r0 += BATCH) {
                float x[BATCH][2];
#pragma unroll
                for (int r = 0; r < BATCH && r0 + r < PER; ++r) {
                    const int i = min((int)threadIdx.x + (r0 + r) * kThreads, NPR - 1);
                    const int row = i / C::NPAIR, j = i % C::NPAIR;
                    x[r][0] = st[row * G::CPITCH + C::P0 + 2 * j];
                    x[r][1] = st[row * G::CPITCH + C::P0 + 2 * j + 1];
                }
#pragma unroll
                for (int r = 0; r < BATCH && r0 + r < PER; ++r) {
                    const int i = (int)threadIdx.x + (r0 + r) * kThreads;
                    if (i < NPR) {
                        const int row = i / C::NPAIR, j = i % C::NPAIR;
                        unsigned h, lo;
                        split2<PART>(x[r][0], x[r][1], sigma, &h, &lo);
                        *reinterpret_cast<u2v *>(conv + (row * C::ROWC + C::pos(j)) * 4) = u2v{h, lo};
                    }
                }
            }
        };
        // the converted plane -> B registers: one 8-byte read per register
        auto gather = [&](auto buf, int l) {
            constexpr int PB = decltype(buf)::value;
            const char *tb = conv + tbo;
#pragma unroll
            for (int c = 0; c < CPP; ++c)
#pragma unroll
                for (int v = 0; v < VPK; ++v) {
                    const u2v w = *reinterpret_cast<const u2v *>(tb + plane_off<VPK>(off2[c], v, l));
                    bh[PB][c][v] = w.x;
                    bl[PB][c][v] = w.y;
                }
        };
        wait_vmcnt<P::W0>();
        __builtin_amdgcn_s_barrier();
        convert(0);
        lds_publish();
        gather(std::integral_constant<int, 0>{}, 0);
        auto step = [&](auto phase, int l) {
            constexpr int S = decltype(phase)::value;   // l % (NB * NZ)
            constexpr int R = S % NZ, PB = S % 2;
            if (l < P::STEADY) wait_vmcnt<P::WL>();
            else wait_vmcnt<P::WS>();
            // every wave's transfers of plane l + 1 have landed, and every
            // wave is done with the converted plane l (gathered a step
            // earlier) and plane l - 1's slot, which the next issue refills
            __builtin_amdgcn_s_barrier();
            issue(l + NP - 1);
            // plane l + 1 converted, then into B registers (past the last
            // plane this reads the repeated last plane, unused), while plane
            // l, gathered one step earlier, is multiplied by every offset
            convert(l + 1);
            lds_publish();
            constexpr int CUR = PB % NB;
            if constexpr (NB == 2) gather(std::integral_constant<int, 1 - PB>{}, l + 1);
#pragma unroll
            for (int c = 0; c < CPP; ++c) {
#pragma unroll
                for (int pz = 0; pz < NZ; ++pz)
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb) {
                        const int kc = pz * CPP + c, i = (NZ - 1 - pz + R) % NZ;
                        accm[i][mb] = mma<MODE, PART>(ahi[mb][kc], bh[CUR][c], accm[i][mb], aidx[mb][kc]);
                        acc1[i][mb] = mma<MODE, PART>(ahi[mb][kc], bl[CUR][c], acc1[i][mb], aidx[mb][kc]);
                    }
#pragma unroll
                for (int pz = 0; pz < NZ; ++pz)
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb) {
                        const int kc = pz * CPP + c, i = (NZ - 1 - pz + R) % NZ;
                        acc1[i][mb] = mma<MODE, PART>(alo[mb][kc], bh[CUR][c], acc1[i][mb], aidx[mb][kc]);
                    }
            }
            if constexpr (NB == 1) gather(std::integral_constant<int, 0>{}, l + 1);
            // output plane z0 + l - 2*RAD (slot R) is complete
            if (l >= 2 * RAD) {
                const int zo = z0 + l - 2 * RAD;
                float *out = static_cast<float *>(g.out) + ((size_t)zo * g.ny + Y0) * g.nx;
                const __amdgpu_buffer_rsrc_t orsrc = uniform_rsrc(out, rows_left * g.nx * 4);
                // band points (fused zero halo) are left to the band pass
                const bool plane_ok = !BAND || (zo >= bnd && zo < g.nz - bnd);
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    const int o = mb * 16 + 4 * q;
                    const int gyr = srow0 + o / R1;
                    const int gx = xbase + o % R1;
                    float ys[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) ys[i] = accm[R][mb][i] + acc1[R][mb][i] * inv_sigma;
                    const bool row_ok =
                        gyr < rows_left && plane_ok && (!BAND || (Y0 + gyr >= bnd && Y0 + gyr < g.ny - bnd));
                    // the band's columns: kBandX0 a side (whole groups of
                    // four on rows of a multiple of 4 values)
                    const int xlo = BAND ? kBandX0 : 0, xhi = BAND ? g.nx - kBandX0 : g.nx;
                    if constexpr (VEC) {
                        const u4v yv = {__float_as_uint(ys[0]), __float_as_uint(ys[1]), __float_as_uint(ys[2]),
                                        __float_as_uint(ys[3])};
                        const bool whole = gx >= xlo && gx + 4 <= xhi;
                        const unsigned o4 = row_ok && whole ? (unsigned)(gyr * g.nx + gx) * 4u : kOob;
                        __builtin_amdgcn_raw_buffer_store_b128(yv, orsrc, o4, 0, 0);
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const unsigned o1 =
                                row_ok && gx + i >= xlo && gx + i < xhi ? (unsigned)(gyr * g.nx + gx + i) * 4u : kOob;
                            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(ys[i]), orsrc, o1, 0, 0);
                        }
                    }
                }
            }
            // slot R starts the newest output plane
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                accm[R][mb] = f4{0.f, 0.f, 0.f, 0.f};
                acc1[R][mb] = f4{0.f, 0.f, 0.f, 0.f};
            }
        };
#pragma unroll 1
        // unrolled so that the accumulator rotation (and the choice of B
        // set) is a renaming
        for (int l0 = 0; l0 < nload; l0 += NB * NZ) unroll_steps<0, NB * NZ>(step, l0, nload);
        // the ring is refilled by the next item: let this item's transfers
        // (including the clamped ones past its last plane) land and every
        // wave finish reading first
        wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
    }
    if constexpr (BAND) band_share3(p, blockIdx.x, nwg, reinterpret_cast<float *>(lds));
}

// Direct 3-D sweep on the vector ALUs (the same-box baseline without the
// matrix product), fed by the same z-march pipeline: thread t computes column
// t % 256 of the 256 x 16 item, rows 8 (t / 256) .. + 7.  Each input plane
// adds its contributions to the 2r+1 output planes it feeds (rotating
// accumulators, as in the matrix kernel), one slab column in registers at a
// time, with FP32 fused multiply-adds and coefficients from an LDS copy.
constexpr int kD3Rows = 8;   // output rows per thread

template <int RAD, bool VEC, int BC, bool BAND>
__global__ __launch_bounds__(kThreads, 1) void k_lds3d(MmaArgs p) {
    using G = Mma3Geom<8, 4, RAD>;
    using P = Pipe3<8, 4, RAD, VEC>;
    constexpr int NP = G::NP;
    constexpr int NZ = 2 * RAD + 1;
    constexpr int NR = kD3Rows + 2 * RAD;           // slab rows a thread reads
    // waits for plane l at step l, as in the first form of the matrix kernel
    // pipeline: loads of the NP-2 planes after it and the stores (one per
    // output row of a thread) of the NP-1 steps since
    constexpr int WL = (NP - 2) * P::D;
    constexpr int WS = (NP - 2) * P::D + (NP - 1) * kD3Rows;
    constexpr int STEADY = 2 * RAD + NP - 1;
    __shared__ __attribute__((aligned(16))) char lds[NP * G::PLANE_BYTES];
    __shared__ float wl[NZ * NZ * NZ];
    const unsigned lds0 = lds_addr_of(lds);
    const float *zf = static_cast<const float *>(p.zeros);
    const int bnd = BAND ? p.edge_rad * (p.edge_steps - 1) : 0;

    const int nxcd = p.nxcd;
    const int nwg = gridDim.x;
    const int xcd = blockIdx.x % nxcd;
    const int stride = nwg / nxcd + (xcd < nwg % nxcd ? 1 : 0);
    const int before = xcd * (nwg / nxcd) + min(xcd, nwg % nxcd);
    const int range_begin = (int)((long long)p.total_items * before / nwg);
    const int range_end = (int)((long long)p.total_items * (before + stride) / nwg);
    const int first = range_begin + blockIdx.x / nxcd;
    for (int i = threadIdx.x; i < NZ * NZ * NZ; i += kThreads) wl[i] = p.w[i];
    // the copy's global loads are the only VMEM loads the compiler tracks
    wait_vmcnt<0>();
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = threadIdx.x % kBandX;
    const int y0 = (threadIdx.x / kBandX) * kD3Rows;
    unsigned row_lds[P::DRW];
#pragma unroll
    for (int d = 0; d < P::DRW; ++d) row_lds[d] = min(wave + d * kWaves, G::SROWS - 1) * G::CPITCH * 4;

#pragma unroll 1
    for (int it = first; it < range_end; it += stride) {
        int j = 0;
        for (int t = 1; t < p.njobs; ++t) j += it >= p.job[t].item0 ? 1 : 0;
        const MmaJob g = p.job[j];
        const int nbands = (g.nx + kBandX - 1) / kBandX, nrb = (g.ny + G::WGH - 1) / G::WGH;
        int local = it - g.item0;
        const int X0 = __builtin_amdgcn_readfirstlane((local % nbands) * kBandX);
        local /= nbands;
        const int Y0 = __builtin_amdgcn_readfirstlane((local % nrb) * G::WGH);
        const int z0 = __builtin_amdgcn_readfirstlane((local / nrb) * g.zc);
        const int nzc = min(g.zc, g.nz - z0);
        const int nload = nzc + 2 * RAD;
        int row_off[P::DRW];
#pragma unroll
        for (int d = 0; d < P::DRW; ++d) {
            const int gy = wrap<BC>(Y0 - RAD + min(wave + d * kWaves, G::SROWS - 1), g.ny);
            row_off[d] = (BC != kBcZero || (gy >= 0 && gy < g.ny)) ? gy * g.nx : -1;
        }
        auto issue = [&](int l) {
            const int zz = wrap<BC>(z0 - RAD + min(l, nload - 1), g.nz);
            issue_plane<8, 4, RAD, VEC, BC>(g, zf, lds0 + (l % NP) * G::PLANE_BYTES, row_off, row_lds, X0, zz);
        };
#pragma unroll 1
        for (int l = 0; l < NP - 1; ++l) issue(l);
        const int rows_left = min(G::WGH, g.ny - Y0);
        const int gx = X0 + c;
        // output plane z0 + l - 2*RAD + i accumulates at step l in slot (i + l) % NZ
        float acc[NZ][kD3Rows];
#pragma unroll
        for (int i = 0; i < NZ; ++i)
#pragma unroll
            for (int y = 0; y < kD3Rows; ++y) acc[i][y] = 0.f;
        auto step = [&](auto rot, int l) {
            constexpr int R = decltype(rot)::value;   // l % NZ
            if (l < STEADY) wait_vmcnt<WL>();
            else wait_vmcnt<WS>();
            __builtin_amdgcn_s_barrier();
            issue(l + NP - 1);
            const float *sl = reinterpret_cast<const float *>(lds + (l % NP) * G::PLANE_BYTES);
            // coefficients by LDS broadcast where they are used (the empty
            // asm keeps the compiler from hoisting all of them)
            int wbase = 0;
            asm volatile("" : "+v"(wbase));
            const float *w = wl + wbase;
#pragma unroll
            for (int dx = 0; dx < NZ; ++dx) {
                int col = G::HL - RAD + c + dx;
                asm volatile("" : "+v"(col));
                float v[NR];
#pragma unroll
                for (int ry = 0; ry < NR; ++ry) v[ry] = sl[(y0 + ry) * G::CPITCH + col];
                // input plane z0 - RAD + l is plane offset 2*RAD - i of
                // logical output i
#pragma unroll
                for (int i = 0; i < NZ; ++i) {
                    const int sidx = (i + R) % NZ, pz = 2 * RAD - i;
#pragma unroll
                    for (int dy = 0; dy < NZ; ++dy) {
                        const float wc = w[(pz * NZ + dy) * NZ + dx];
#pragma unroll
                        for (int y = 0; y < kD3Rows; ++y) acc[sidx][y] = fmaf(wc, v[y + dy], acc[sidx][y]);
                    }
                }
#pragma unroll
                for (int i = 0; i < NZ; ++i)
#pragma unroll
                    for (int y = 0; y < kD3Rows; ++y) asm volatile("" : "+v"(acc[i][y]));
            }
            if (l >= 2 * RAD) {
                const int zo = z0 + l - 2 * RAD;
                float *out = static_cast<float *>(g.out) + ((size_t)zo * g.ny + Y0) * g.nx;
                const __amdgpu_buffer_rsrc_t orsrc = uniform_rsrc(out, rows_left * g.nx * 4);
                // band points (fused zero halo) are left to the band pass
                const bool col_ok =
                    BAND ? zo >= bnd && zo < g.nz - bnd && gx >= kBandX0 && gx < g.nx - kBandX0 : gx < g.nx;
#pragma unroll
                for (int y = 0; y < kD3Rows; ++y) {
                    const bool row_ok = y0 + y < rows_left && (!BAND || (Y0 + y0 + y >= bnd && Y0 + y0 + y < g.ny - bnd));
                    const unsigned o = row_ok && col_ok ? (unsigned)((y0 + y) * g.nx + gx) * 4u : kOob;
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[R][y]), orsrc, o, 0, 0);
                }
            }
#pragma unroll
            for (int y = 0; y < kD3Rows; ++y) acc[R][y] = 0.f;
        };
#pragma unroll 1
        for (int l0 = 0; l0 < nload; l0 += NZ) unroll_steps<0, NZ>(step, l0, nload);
        wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
    }
    if constexpr (BAND) band_share3(p, blockIdx.x, nwg, reinterpret_cast<float *>(lds));
}

template <int RAD, bool VEC, int BC>
static hipError_t launch_lds3d_bc(const MmaArgs &a, int cus, int xcds, hipStream_t s) {
    MmaArgs b = a;
    b.nxcd = xcds;
    const int g = a.total_items < cus ? a.total_items : cus;
    if constexpr (BC == kBcZero && RAD >= 2) {
        if (a.edge_steps > 1) {
            hipLaunchKernelGGL((k_lds3d<RAD, VEC, BC, true>), dim3(g), dim3(kThreads), 0, s, b);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_lds3d<RAD, VEC, BC, false>), dim3(g), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

template <int R1, int R2, int KC, int RAD, int MODE, int PART, bool VEC, int BC>
static hipError_t launch3_bc(const MmaArgs &a, int cus, int xcds, hipStream_t s) {
    MmaArgs b = a;
    b.nxcd = xcds;
    const int g = a.total_items < cus ? a.total_items : cus;
    // fused zero-halo launches compose radius-1 sweeps: radius 2 and up
    if constexpr (BC == kBcZero && RAD >= 2) {
        if (a.edge_steps > 1) {
            hipLaunchKernelGGL((k_mma3d<R1, R2, KC, RAD, MODE, PART, VEC, BC, true>), dim3(g), dim3(kThreads), 0, s,
                               b);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_mma3d<R1, R2, KC, RAD, MODE, PART, VEC, BC, false>), dim3(g), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

// Number the jobs' work items (each job's z range split into chunks so that
// the launch has about one item per CU or more), then pick the variant.
template <int R1, int R2, int KC, int RAD, int MODE, int PART>
static hipError_t launch_mma3d(MmaArgs &a, hipStream_t s) {
    using G = Mma3Geom<R1, R2, RAD>;
    if (a.njobs < 1 || a.njobs > kMaxJobs) return hipErrorInvalidValue;
    int cus = 0, xcds = 0;
    if (const hipError_t e = device_shape(&cus, &xcds); e != hipSuccess) return e;
    int columns = 0;
    for (int j = 0; j < a.njobs; ++j)
        columns += ((a.job[j].nx + kBandX - 1) / kBandX) * ((a.job[j].ny + G::WGH - 1) / G::WGH);
    const int chunks = columns >= cus ? 1 : (cus + columns - 1) / columns;
    int items = 0;
    bool vec = true, wrap1 = true;
    for (int j = 0; j < a.njobs; ++j) {
        MmaJob &g = a.job[j];
        g.zc = (g.nz + chunks - 1) / chunks;
        g.item0 = items;
        items += ((g.nx + kBandX - 1) / kBandX) * ((g.ny + G::WGH - 1) / G::WGH) * ((g.nz + g.zc - 1) / g.zc);
        vec = vec && (g.nx & 3) == 0;
        wrap1 = wrap1 && g.ny >= G::SROWS && g.nx >= kBandX + 2 * RAD && g.nz >= 2 * RAD + 1;
    }
    a.total_items = items;
    if (items == 0) return hipSuccess;
    if (vec) {
        if (!a.periodic) return launch3_bc<R1, R2, KC, RAD, MODE, PART, true, kBcZero>(a, cus, xcds, s);
        if (wrap1) return launch3_bc<R1, R2, KC, RAD, MODE, PART, true, kBcWrap1>(a, cus, xcds, s);
        return launch3_bc<R1, R2, KC, RAD, MODE, PART, true, kBcWrapN>(a, cus, xcds, s);
    }
    if (!a.periodic) return launch3_bc<R1, R2, KC, RAD, MODE, PART, false, kBcZero>(a, cus, xcds, s);
    if (wrap1) return launch3_bc<R1, R2, KC, RAD, MODE, PART, false, kBcWrap1>(a, cus, xcds, s);
    return launch3_bc<R1, R2, KC, RAD, MODE, PART, false, kBcWrapN>(a, cus, xcds, s);
}

#define SS_MMA3(R1, R2, KC, RAD, MODE, PART)                                                        \
    {{R1, R2, KC, RAD, MODE, PART, kStateF32},                                                      \
     &launch_mma3d<R1, R2, KC, RAD, MODE, PART>, Mma3Geom<R1, R2, RAD>::WGH, Conv3Geom<R1, R2, RAD>::ROWC, \
     Conv3Geom<R1, R2, RAD>::PW, Conv3Geom<R1, R2, RAD>::PADG}

// Radius 1 (k = 3) at tile (8,4): every plane has 60 staircase columns,
// padded to one 64-wide sparse chunk (K 192) or two 32-wide dense chunks
// (K 192).  Radius 2 (two radius-1 sweeps composed) at tile (8,2): a plane
// has 72 staircase columns; the union of the planes' used columns takes two
// sparse or three dense chunks a plane for the 27-point box (K 640 / 480)
// and one sparse or two dense chunks for the 7-point star, whose composed
// planes use at most the 13 points of a radius-2 diamond (K 320 / 320).
static const MmaEntry kTable3[] = {
    SS_MMA3(8, 4, 3, 1, kSparse, kPartF16),   SS_MMA3(8, 4, 6, 1, kDense, kPartF16),
    SS_MMA3(8, 4, 3, 1, kSparse, kPartBF16),  SS_MMA3(8, 4, 6, 1, kDense, kPartBF16),
    SS_MMA3(8, 2, 10, 2, kSparse, kPartF16),  SS_MMA3(8, 2, 15, 2, kDense, kPartF16),
    SS_MMA3(8, 2, 5, 2, kSparse, kPartF16),   SS_MMA3(8, 2, 10, 2, kDense, kPartF16),
    SS_MMA3(8, 2, 10, 2, kSparse, kPartBF16), SS_MMA3(8, 2, 15, 2, kDense, kPartBF16),
    SS_MMA3(8, 2, 5, 2, kSparse, kPartBF16),  SS_MMA3(8, 2, 10, 2, kDense, kPartBF16),
};

MmaLaunch find_mma3d(const MmaKey &k) {
    for (const MmaEntry &e : kTable3)
        if (e.key.r1 == k.r1 && e.key.r2 == k.r2 && e.key.kc == k.kc && e.key.rad == k.rad &&
            e.key.mode == k.mode && e.key.part == k.part)
            return e.fn;
    return nullptr;
}

bool mma3d_geometry(const MmaKey &k, int *wgh, int *row, int *pw, int *padg) {
    for (const MmaEntry &e : kTable3)
        if (e.key.r1 == k.r1 && e.key.r2 == k.r2 && e.key.kc == k.kc && e.key.rad == k.rad &&
            e.key.mode == k.mode && e.key.part == k.part) {
            *wgh = e.wgh;
            *row = e.row;
            *pw = e.pw;
            *padg = e.padg;
            return true;
        }
    return false;
}

// Number a launch's work items as for the matrix kernels (z chunks so that
// there is about one item per CU or more) and pick the variant.
template <int RAD>
static hipError_t launch_lds3d(MmaArgs &a, hipStream_t s) {
    using G = Mma3Geom<8, 4, RAD>;
    if (a.njobs < 1 || a.njobs > kMaxJobs) return hipErrorInvalidValue;
    int cus = 0, xcds = 0;
    if (const hipError_t e = device_shape(&cus, &xcds); e != hipSuccess) return e;
    int columns = 0;
    for (int j = 0; j < a.njobs; ++j)
        columns += ((a.job[j].nx + kBandX - 1) / kBandX) * ((a.job[j].ny + G::WGH - 1) / G::WGH);
    const int chunks = columns >= cus ? 1 : (cus + columns - 1) / columns;
    int items = 0;
    bool vec = true, wrap1 = true;
    for (int j = 0; j < a.njobs; ++j) {
        MmaJob &g = a.job[j];
        g.zc = (g.nz + chunks - 1) / chunks;
        g.item0 = items;
        items += ((g.nx + kBandX - 1) / kBandX) * ((g.ny + G::WGH - 1) / G::WGH) * ((g.nz + g.zc - 1) / g.zc);
        vec = vec && (g.nx & 3) == 0;
        wrap1 = wrap1 && g.ny >= G::SROWS && g.nx >= kBandX + 2 * RAD && g.nz >= 2 * RAD + 1;
    }
    a.total_items = items;
    if (items == 0) return hipSuccess;
    if (vec) {
        if (!a.periodic) return launch_lds3d_bc<RAD, true, kBcZero>(a, cus, xcds, s);
        if (wrap1) return launch_lds3d_bc<RAD, true, kBcWrap1>(a, cus, xcds, s);
        return launch_lds3d_bc<RAD, true, kBcWrapN>(a, cus, xcds, s);
    }
    if (!a.periodic) return launch_lds3d_bc<RAD, false, kBcZero>(a, cus, xcds, s);
    if (wrap1) return launch_lds3d_bc<RAD, false, kBcWrap1>(a, cus, xcds, s);
    return launch_lds3d_bc<RAD, false, kBcWrapN>(a, cus, xcds, s);
}

MmaLaunch find_lds_direct3d(int rad) {
    switch (rad) {
        case 1: return &launch_lds3d<1>;
        case 2: return &launch_lds3d<2>;
    }
    return nullptr;
}

int mma3d_keys(int rad, int mode, int part, MmaKey *out, int max) {
    int n = 0;
    for (const MmaEntry &e : kTable3)
        if (e.key.rad == rad && e.key.mode == mode && e.key.part == part && n < max) out[n++] = e.key;
    return n;
}

}  // namespace ss
