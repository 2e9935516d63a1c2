// 3-D stencil sweep as a structured-sparse (or dense) matrix product on
// gfx950 matrix cores, FP32 state split into hi + lo parts as it is gathered.
//
// The 3-D staircase matrix A' has one block level more than in 2-D: a patch
// is 2r+1 z planes of the 2-D patch, and each output tile of r2 x r1 points
// in one z plane uses all of them.  The matching runs per plane (the planes'
// columns never share a 4-group here), and every plane's K columns are
// padded to whole MMA chunks, so that a chunk gathers from a single input
// plane.  A work item is a 256 x WGH column of the grid over ZC planes; the
// workgroup streams the input planes through a ring of LDS slabs filled by
// LDS DMA several planes ahead.  Each input plane is gathered into B
// registers once and multiplied by the A blocks of all 2r+1 plane offsets,
// accumulating into the 2r+1 output planes it contributes to; the oldest of
// those is complete after the plane and is stored.
#include <hip/hip_runtime.h>

#include "mma2d_impl.hpp"

namespace ss {

template <int R1, int R2, int RAD, bool VEC>
struct Pipe3 {
    using G = Mma3Geom<R1, R2, RAD>;
    static constexpr int DRW = (G::SROWS + kWaves - 1) / kWaves;   // rows each wave loads per plane
    static constexpr int DMA_PER_ROW = VEC ? 1 : kBandX / 64;
    static constexpr int D1 = DRW * DMA_PER_ROW;                   // VMEM loads per plane, waves 1..7
    static constexpr int D0 = D1 + G::HOPS;                        // ... wave 0 (also the halo)
    static constexpr int M = G::MB * (VEC ? 1 : 4);                // VMEM stores per output plane
    static constexpr int A = 2 * RAD;                              // steps before the first store
    // VMEM operations issued after load p when step p consumes it: loads
    // 0..NP-2 are issued before step 0, step j issues load j+NP-1 and then,
    // from step A on, the stores of one output plane; S = min(max(p-A, 0),
    // NP-1) counts the steps with stores among those that follow load p
    template <int D, int S>
    static constexpr int W = (G::NP - 2) * D + S * M;
};

template <int D, int R1, int R2, int RAD, bool VEC>
__device__ inline void wait_step3(int p) {
    using P = Pipe3<R1, R2, RAD, VEC>;
    constexpr int NP = Mma3Geom<R1, R2, RAD>::NP;
    const int st = min(max(p - P::A, 0), NP - 1);
    static_assert(NP <= 8, "wait table covers up to 8 ring slots");
    switch (st) {
        case 0: wait_vmcnt<P::template W<D, 0>>(); break;
        case 1: wait_vmcnt<P::template W<D, 1>>(); break;
        case 2: wait_vmcnt<P::template W<D, 2>>(); break;
        case 3: wait_vmcnt<P::template W<D, 3>>(); break;
        case 4: wait_vmcnt<P::template W<D, 4>>(); break;
        case 5: wait_vmcnt<P::template W<D, 5>>(); break;
        case 6: wait_vmcnt<P::template W<D, 6>>(); break;
        default: wait_vmcnt<P::template W<D, 7>>(); break;
    }
}

// Issue the transfers of input plane z (already wrapped, or outside the grid
// with a zero halo) into a ring slot: every row of the slab by every wave
// (rows clamped, so all waves issue DRW rows), halo columns by wave 0.
template <int R1, int R2, int RAD, bool VEC, int BC>
__device__ inline void issue_plane(const MmaArgs &p, const MmaJob &g, char *slab, unsigned *strip, int X0,
                                   int Y0, int z) {
    using G = Mma3Geom<R1, R2, RAD>;
    using P = Pipe3<R1, R2, RAD, VEC>;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    X0 = __builtin_amdgcn_readfirstlane(X0);
    Y0 = __builtin_amdgcn_readfirstlane(Y0);
    z = __builtin_amdgcn_readfirstlane(z);
    const bool z_ok = BC != kBcZero || (z >= 0 && z < g.nz);
    const float *in = static_cast<const float *>(g.in) + (size_t)(z_ok ? z : 0) * g.ny * g.nx;
    const float *zf = static_cast<const float *>(p.zeros);
#pragma unroll
    for (int d = 0; d < P::DRW; ++d) {
        const int r = min(wave + d * kWaves, G::SROWS - 1);
        const int gy = wrap<BC>(Y0 - RAD + r, g.ny);
        const bool row_ok = BC != kBcZero || (z_ok && gy >= 0 && gy < g.ny);
        const unsigned dst = lds_addr_of(reinterpret_cast<float *>(slab) + r * G::CPITCH + G::HL);
        if constexpr (VEC) {
            const int gx = wrap<BC>(X0 + 4 * lane, g.nx);
            const bool ok = BC != kBcZero || (row_ok && gx < g.nx);
            lds_dma16(ok ? in + (size_t)gy * g.nx + gx : zf + 4 * lane, dst);
        } else {
#pragma unroll
            for (int h = 0; h < P::DMA_PER_ROW; ++h) {
                const int gx = wrap<BC>(X0 + 64 * h + lane, g.nx);
                const bool ok = BC != kBcZero || (row_ok && gx < g.nx);
                lds_dma4(ok ? in + (size_t)gy * g.nx + gx : zf + lane, dst + 256 * h);
            }
        }
    }
    if (wave == 0) {
#pragma unroll
        for (int h = 0; h < G::HOPS; ++h) {
            const int e = min(h * 64 + lane, G::NHALO - 1);
            const int r = e / (2 * RAD), j = e % (2 * RAD);
            const int gy = wrap<BC>(Y0 - RAD + r, g.ny);
            const int gx = wrap<BC>(j < RAD ? X0 - RAD + j : X0 + kBandX + (j - RAD), g.nx);
            const bool ok = BC != kBcZero || (z_ok && gy >= 0 && gy < g.ny && gx >= 0 && gx < g.nx);
            lds_dma4(ok ? in + (size_t)gy * g.nx + gx : zf + lane, lds_addr_of(strip + h * 64));
        }
    }
}

template <int R1, int R2, int RAD>
__device__ inline void put_halo3(char *slab, const unsigned *strip) {
    using G = Mma3Geom<R1, R2, RAD>;
    for (int e = threadIdx.x; e < G::NHALO; e += kThreads) {
        const int r = e / (2 * RAD), j = e % (2 * RAD);
        const int c = j < RAD ? G::HL - RAD + j : G::HL + kBandX + (j - RAD);
        reinterpret_cast<unsigned *>(slab)[r * G::CPITCH + c] = strip[e];
    }
}

template <int R1, int R2, int KC, int RAD, int MODE, int PART, bool VEC, int BC>
__global__ __launch_bounds__(kThreads, 1) void k_mma3d(MmaArgs p) {
    using G = Mma3Geom<R1, R2, RAD>;
    using P = Pipe3<R1, R2, RAD, VEC>;
    constexpr int MB = G::MB;
    constexpr int VPK = (MODE == kSparse) ? 8 : 4;
    constexpr int NP = G::NP;
    constexpr int NZ = 2 * RAD + 1;          // plane offsets of the stencil
    constexpr int CPP = KC / NZ;             // K chunks per input plane
    static_assert(CPP * NZ == KC, "chunks must not straddle planes");
    __shared__ __attribute__((aligned(16))) char lds[NP * G::SLOT];
    auto slab = [&](int i) { return lds + i * G::PLANE_BYTES; };
    auto strip = [&](int i) { return reinterpret_cast<unsigned *>(lds + NP * G::PLANE_BYTES) + i * G::HSTRIP; };

    const float sigma = 1.0f / p.inv_sigma;
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
    const int wave = threadIdx.x >> 6;
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

#pragma unroll 1
    for (int it = first; it < range_end; it += stride) {
        // item -> job, band, row block, z chunk
        int j = 0;
        for (int t = 1; t < p.njobs; ++t) j += it >= p.job[t].item0 ? 1 : 0;
        const MmaJob &g = p.job[j];
        const int nbands = (g.nx + kBandX - 1) / kBandX, nrb = (g.ny + G::WGH - 1) / G::WGH;
        int local = it - g.item0;
        const int X0 = (local % nbands) * kBandX;
        local /= nbands;
        const int Y0 = (local % nrb) * G::WGH;
        const int z0 = (local / nrb) * g.zc;
        const int nzc = min(g.zc, g.nz - z0);
        const int nload = nzc + 2 * RAD;   // input planes z0-RAD .. z0+nzc-1+RAD
        auto issue = [&](int l) {
            const int zz = wrap<BC>(z0 - RAD + min(l, nload - 1), g.nz);
            issue_plane<R1, R2, RAD, VEC, BC>(p, g, slab(l % NP), strip(l % NP), X0, Y0, zz);
        };
#pragma unroll 1
        for (int l = 0; l < NP - 1; ++l) issue(l);
        const int rows_left = min(G::WGH, g.ny - Y0);
        const int xbase = X0 + nbc * 128 + tx_t * R1;
        // acc[i] accumulates output plane z0 + (l - 2*RAD + i) at step l
        // hi*hi, hi*lo and lo*hi accumulate separately
        f4 accm[NZ][MB], acc1[NZ][MB], acc2[NZ][MB];
#pragma unroll
        for (int i = 0; i < NZ; ++i)
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                accm[i][mb] = f4{0.f, 0.f, 0.f, 0.f};
                acc1[i][mb] = f4{0.f, 0.f, 0.f, 0.f};
                acc2[i][mb] = f4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll 1
        for (int l = 0; l < nload; ++l) {
            if (wave == 0) wait_step3<P::D0, R1, R2, RAD, VEC>(l);
            else wait_step3<P::D1, R1, R2, RAD, VEC>(l);
            __builtin_amdgcn_s_barrier();
            put_halo3<R1, R2, RAD>(slab(l % NP), strip(l % NP));
            __builtin_amdgcn_s_waitcnt(0xC07F);
            __builtin_amdgcn_s_barrier();
            issue(l + NP - 1);
            // input plane l: once into B registers, times every plane offset
            const char *tb =
                slab(l % NP) + (srow0 * G::CPITCH + (G::HL - RAD) + nbc * 128 + tx_t * R1) * 4;
#pragma unroll
            for (int c = 0; c < CPP; ++c) {
                unsigned bh[VPK], bl[VPK];
#pragma unroll
                for (int v = 0; v < VPK; ++v) {
                    const float *src = reinterpret_cast<const float *>(tb + gather_off<VPK>(off2[c], v));
                    split2<PART>(src[0], src[1], sigma, &bh[v], &bl[v]);
                }
#pragma unroll
                for (int pz = 0; pz < NZ; ++pz)
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb) {
                        const int kc = pz * CPP + c, i = NZ - 1 - pz;
                        accm[i][mb] = mma<MODE, PART>(ahi[mb][kc], bh, accm[i][mb], aidx[mb][kc]);
                        acc1[i][mb] = mma<MODE, PART>(ahi[mb][kc], bl, acc1[i][mb], aidx[mb][kc]);
                        acc2[i][mb] = mma<MODE, PART>(alo[mb][kc], bh, acc2[i][mb], aidx[mb][kc]);
                    }
            }
            // output plane z0 + l - 2*RAD is complete
            if (l >= 2 * RAD) {
                float *out = static_cast<float *>(g.out) + ((size_t)(z0 + l - 2 * RAD) * g.ny + Y0) * g.nx;
                const __amdgpu_buffer_rsrc_t orsrc = uniform_rsrc(out, rows_left * g.nx * 4);
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    const int o = mb * 16 + 4 * q;
                    const int gyr = srow0 + o / R1;
                    const int gx = xbase + o % R1;
                    float ys[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) ys[i] = accm[0][mb][i] + (acc1[0][mb][i] + acc2[0][mb][i]) * p.inv_sigma;
                    const bool row_ok = gyr < rows_left;
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
#pragma unroll
            for (int i = 0; i + 1 < NZ; ++i)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    accm[i][mb] = accm[i + 1][mb];
                    acc1[i][mb] = acc1[i + 1][mb];
                    acc2[i][mb] = acc2[i + 1][mb];
                }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                accm[NZ - 1][mb] = f4{0.f, 0.f, 0.f, 0.f};
                acc1[NZ - 1][mb] = f4{0.f, 0.f, 0.f, 0.f};
                acc2[NZ - 1][mb] = f4{0.f, 0.f, 0.f, 0.f};
            }
        }
        // the ring is refilled by the next item: let this item's transfers
        // (including the clamped ones past its last plane) land and every
        // wave finish reading first
        wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
    }
}

template <int R1, int R2, int KC, int RAD, int MODE, int PART, bool VEC, int BC>
static hipError_t launch3_bc(const MmaArgs &a, int cus, int xcds, hipStream_t s) {
    MmaArgs b = a;
    b.nxcd = xcds;
    const int g = a.total_items < cus ? a.total_items : cus;
    hipLaunchKernelGGL((k_mma3d<R1, R2, KC, RAD, MODE, PART, VEC, BC>), dim3(g), dim3(kThreads), 0, s, b);
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
     &launch_mma3d<R1, R2, KC, RAD, MODE, PART>, Mma3Geom<R1, R2, RAD>::WGH, Mma3Geom<R1, R2, RAD>::CPITCH}

// Radius 1 (k = 3) at tile (8,4): every plane has 60 staircase columns,
// padded to one 64-wide sparse chunk (K 192) or two 32-wide dense chunks
// (K 192).
static const MmaEntry kTable3[] = {
    SS_MMA3(8, 4, 3, 1, kSparse, kPartF16),  SS_MMA3(8, 4, 6, 1, kDense, kPartF16),
    SS_MMA3(8, 4, 3, 1, kSparse, kPartBF16), SS_MMA3(8, 4, 6, 1, kDense, kPartBF16),
};

MmaLaunch find_mma3d(const MmaKey &k) {
    for (const MmaEntry &e : kTable3)
        if (e.key.r1 == k.r1 && e.key.r2 == k.r2 && e.key.kc == k.kc && e.key.rad == k.rad &&
            e.key.mode == k.mode && e.key.part == k.part)
            return e.fn;
    return nullptr;
}

bool mma3d_geometry(const MmaKey &k, int *wgh, int *row) {
    for (const MmaEntry &e : kTable3)
        if (e.key.r1 == k.r1 && e.key.r2 == k.r2 && e.key.kc == k.kc && e.key.rad == k.rad &&
            e.key.mode == k.mode && e.key.part == k.part) {
            *wgh = e.wgh;
            *row = e.row;
            return true;
        }
    return false;
}

int mma3d_keys(int rad, int mode, int part, MmaKey *out, int max) {
    int n = 0;
    for (const MmaEntry &e : kTable3)
        if (e.key.rad == rad && e.key.mode == mode && e.key.part == part && n < max) out[n++] = e.key;
    return n;
}

}  // namespace ss
