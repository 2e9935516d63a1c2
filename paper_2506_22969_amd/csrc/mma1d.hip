// 1-D stencil sweep as a structured-sparse (or dense) matrix product on
// gfx950 matrix cores, FP32 state split into binary16 or bfloat16 hi + lo
// parts as it is gathered (paper Sections 3.1-3.3 with one tile row).
//
// A tile is 16 consecutive outputs (r1 = 16, r2 = 1): A' is the 16 x (15+k)
// band of the coefficients, and sixteen tiles (256 consecutive outputs) form
// the N dimension of one MMA.  The work is a stream: every workgroup stages
// 4096 outputs' inputs (plus 8 on each side) into LDS with 16-byte loads,
// multiplies them out and writes the outputs back 16 bytes per lane, so the
// sweep is bound by HBM like any 1-D stencil.
//
// LDS keeps one padding word after every 16 values: tile n of an MMA starts
// 17n words after tile 0, so the sixteen B columns of a gather fall into
// different banks.  The gather offset of patch column p is then
// p + ((c0 + p) >> 4) for every tile, with c0 = 8 - radius.
//
// The direct engine's 1-D kernel (k_lds1d) shares the staging.  A launch of
// S fused sweeps on a zero-halo grid has one more workgroup, which
// recomputes the points within r(S-1) of either end exactly while the other
// workgroups leave them unwritten.
#include "mma2d_impl.hpp"

namespace ss {
namespace {

constexpr int k1Threads = 256;
constexpr int k1Block = 4096;                   // outputs per workgroup
constexpr int k1Halo = 8;                       // staged inputs on each side
constexpr int k1Span = k1Block + 2 * k1Halo;    // staged inputs
constexpr int k1Words = k1Span + k1Span / 16 + 1;
constexpr int k1PerWave = k1Block / (k1Threads / 64);   // outputs per wave
static_assert(k1PerWave % 256 == 0, "a wave owns whole MMAs");

__device__ inline int skewed(int i) { return i + (i >> 4); }

// Exact values of the points within r(S-1) of either end of every grid after
// S zero-halo sweeps, by threads 0..63 of one workgroup, one point at a time
// per thread: the window of inputs the point depends on is swept S times in
// FP32 (in LDS, shrinking by r on each side per sweep, FMAs in a fixed
// order) with the points outside the grid held at zero.
constexpr int kEdgeWin = 2 * k1Halo + 1;
constexpr int kEdgeLanes = 64;

__device__ inline int band_width(const MmaArgs &p) { return p.edge_rad * (p.edge_steps - 1); }

__device__ inline void end_bands(const MmaArgs &p, float (*buf)[kEdgeWin][kEdgeLanes]) {
    const int lane = threadIdx.x;
    if (lane >= kEdgeLanes) return;
    const int b = band_width(p);
    const int R = p.edge_rad * p.edge_steps;
    const int L = 2 * R + 1, k = 2 * p.edge_rad + 1;
    for (int j = 0; j < p.njobs; ++j) {
        const MmaJob g = p.job[j];
        const int n = g.nx;
        const int lo_count = min(b, n);
        const int count = min(2 * b, n);
        const float *in = static_cast<const float *>(g.in);
        float *out = static_cast<float *>(g.out);
        for (int i = lane; i < count; i += kEdgeLanes) {
            const int pt = i < lo_count ? i : n - (i - lo_count) - 1;
            float(*cur)[kEdgeLanes] = buf[0];
            float(*nxt)[kEdgeLanes] = buf[1];
            for (int w = 0; w < L; ++w) {
                const int gi = pt - R + w;
                cur[w][lane] = (gi >= 0 && gi < n) ? in[gi] : 0.f;
            }
            for (int s = 1; s <= p.edge_steps; ++s) {
                for (int w = s * p.edge_rad; w < L - s * p.edge_rad; ++w) {
                    const int gi = pt - R + w;
                    float acc = 0.f;
                    for (int o = 0; o < k; ++o) acc = __builtin_fmaf(p.edge_w32[o], cur[w + o - p.edge_rad][lane], acc);
                    nxt[w][lane] = (gi >= 0 && gi < n) ? acc : 0.f;
                }
                float(*tmp)[kEdgeLanes] = cur;
                cur = nxt;
                nxt = tmp;
            }
            out[pt] = cur[R][lane];
        }
    }
}

// Stage x[first, first + 4112) into the skewed LDS row: 16-byte loads away
// from the ends, element by element (zero or wrapped) near them.
template <int BC, bool VEC>
__device__ inline void stage_block(const __attribute__((address_space(1))) float *x, int first, int n, float *lds) {
    const int tid = threadIdx.x;
    if (VEC && first >= 0 && first + k1Span <= n) {
        constexpr int NV = k1Span / 4;
        constexpr int PER = (NV + k1Threads - 1) / k1Threads;
        f4 v[PER];
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int i = tid + r * k1Threads;
            if (i < NV) v[r] = *(const __attribute__((address_space(1))) f4 *)(x + first + 4 * i);
        }
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int i = tid + r * k1Threads;
            if (i < NV) {
                // four values of one 16-value run: consecutive words
                float *d = lds + skewed(4 * i);
                d[0] = v[r].x;
                d[1] = v[r].y;
                d[2] = v[r].z;
                d[3] = v[r].w;
            }
        }
    } else {
        for (int i = tid; i < k1Span; i += k1Threads) {
            const int gi = first + i;
            float v = 0.0f;
            if (gi >= 0 && gi < n) v = x[gi];
            else if constexpr (BC != kBcZero) v = x[wrap<kBcWrapN>(gi, n)];
            lds[skewed(i)] = v;
        }
    }
}

template <int KC, int RAD, int MODE, int PART, int BC, bool VEC>
__global__ __launch_bounds__(k1Threads) void k_mma1d(MmaArgs p) {
    static_assert(RAD >= 1 && RAD <= k1Halo, "radius within the staged halo");
    constexpr int VPK = (MODE == kSparse) ? 8 : 4;
    __shared__ __attribute__((aligned(16))) float lds[k1Words];
    static_assert(sizeof(float) * k1Words >= sizeof(float) * 2 * kEdgeWin * kEdgeLanes, "end-band buffers fit");

    // the workgroup after the last block recomputes the end bands
    if (p.edge_w && (int)blockIdx.x == p.total_items) {
        end_bands(p, reinterpret_cast<float(*)[kEdgeWin][kEdgeLanes]>(lds));
        return;
    }

    // the job of this workgroup (jobs' first blocks ascend)
    int j = 0;
    for (int t = 1; t < p.njobs; ++t) j = (int)blockIdx.x >= p.job[t].item0 ? t : j;
    const MmaJob g = p.job[j];
    const int n = g.nx;
    const int base = ((int)blockIdx.x - g.item0) * k1Block;
    // the grid is global memory: say so, so that the loads are global ones
    const __attribute__((address_space(1))) float *x =
        (const __attribute__((address_space(1))) float *)static_cast<const float *>(g.in);
    const int tid = threadIdx.x;

    stage_block<BC, VEC>(x, base - k1Halo, n, lds);

    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int q = lane >> 4;
    const int tile = lane & 15;
    // A fragments and per-lane gather offsets (words from the tile's first
    // patch word; each B register reads two patch columns p, p + 1)
    uint4 ahi[KC], alo[KC];
    unsigned aidx[KC];
    int off[KC][VPK][2];
    constexpr int c0 = k1Halo - RAD;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        ahi[kc] = p.a_hi[kc * 64 + lane];
        alo[kc] = p.a_lo[kc * 64 + lane];
        aidx[kc] = MODE == kSparse ? p.a_idx[kc * 64 + lane] : 0u;
#pragma unroll
        for (int v = 0; v < VPK; ++v) {
            const int pc = p.boff[(kc * 4 + q) * VPK + v] >> 2;
            off[kc][v][0] = pc + ((c0 + pc) >> 4);
            off[kc][v][1] = pc + 1 + ((c0 + pc + 1) >> 4);
        }
    }
    const float sigma = 1.0f / p.inv_sigma;
    const float inv_sigma = p.inv_sigma;
    __syncthreads();

    // outputs of this block that exist, and a store descriptor over them;
    // the end bands of a fused zero-halo launch are left to the last
    // workgroup (outputs [0, lo_end) and [hi_start, n))
    const int valid = min(k1Block, n - base);
    float *out = static_cast<float *>(g.out) + base;
    const __amdgpu_buffer_rsrc_t orsrc = uniform_rsrc(out, valid * 4);
    const int bw = p.edge_w ? band_width(p) : 0;
    const int lo_end = min(bw, n) - base;
    const int hi_start = max(n - bw, min(bw, n)) - base;
    const bool plain = lo_end <= 0 && hi_start >= valid;
#pragma unroll 1
    for (int u = 0; u < k1PerWave / 256; ++u) {
        const int o0 = wave * k1PerWave + u * 256;     // first output of the MMA
        // first patch word of this lane's tile: staged index c0 + o0 + 16 tile
        const float *tb = lds + (c0 + 17 * ((o0 >> 4) + tile));
        f4 accm = {0.f, 0.f, 0.f, 0.f}, acc1 = accm, acc2 = accm;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            unsigned bh[VPK], bl[VPK];
#pragma unroll
            for (int v = 0; v < VPK; ++v) split2<PART>(tb[off[kc][v][0]], tb[off[kc][v][1]], sigma, &bh[v], &bl[v]);
            accm = mma<MODE, PART>(ahi[kc], bh, accm, aidx[kc]);
            acc1 = mma<MODE, PART>(ahi[kc], bl, acc1, aidx[kc]);
            acc2 = mma<MODE, PART>(alo[kc], bh, acc2, aidx[kc]);
        }
        // accumulator rows 4q..4q+3 are outputs o0 + 16 tile + 4q + i
        const int o = o0 + 16 * tile + 4 * q;
        float ys[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) ys[i] = accm[i] + (acc1[i] + acc2[i]) * inv_sigma;
        if (VEC && plain) {
            const u4v yv = {__float_as_uint(ys[0]), __float_as_uint(ys[1]), __float_as_uint(ys[2]),
                            __float_as_uint(ys[3])};
            __builtin_amdgcn_raw_buffer_store_b128(yv, orsrc, o < valid ? (unsigned)o * 4u : kOob, 0, 0);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int oi = o + i;
                const bool keep = oi < valid && oi >= lo_end && oi < hi_start;
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(ys[i]), orsrc, keep ? (unsigned)oi * 4u : kOob,
                                                      0, 0);
            }
        }
    }
}

template <int KC, int RAD, int MODE, int PART>
hipError_t launch_mma1d(MmaArgs &a, hipStream_t s) {
    if (a.njobs < 1 || a.njobs > kMaxJobs) return hipErrorInvalidValue;
    int blocks = 0;
    bool vec = true;
    for (int j = 0; j < a.njobs; ++j) {
        MmaJob &g = a.job[j];
        if (g.nx < 1) return hipErrorInvalidValue;
        g.item0 = blocks;
        blocks += (g.nx + k1Block - 1) / k1Block;
        // 16-byte loads and stores need 16-byte aligned grids of whole float4s
        vec = vec && g.nx % 4 == 0 && ((uintptr_t)g.in % 16) == 0 && ((uintptr_t)g.out % 16) == 0;
    }
    a.total_items = blocks;
    // fused zero-halo sweeps: one more workgroup for the end bands
    if (a.edge_w && (a.edge_steps < 2 || a.edge_rad < 1 || a.edge_rad * a.edge_steps > k1Halo))
        return hipErrorInvalidValue;
    const dim3 grid(blocks + (a.edge_w ? 1 : 0)), block(k1Threads);
    if (a.periodic) {
        if (vec) hipLaunchKernelGGL((k_mma1d<KC, RAD, MODE, PART, kBcWrapN, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_mma1d<KC, RAD, MODE, PART, kBcWrapN, false>), grid, block, 0, s, a);
    } else {
        if (vec) hipLaunchKernelGGL((k_mma1d<KC, RAD, MODE, PART, kBcZero, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_mma1d<KC, RAD, MODE, PART, kBcZero, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

// Direct 1-D sweep from the same staging: each thread sums 16 consecutive
// outputs with FP32 FMAs from the skewed LDS row (threads 17 words apart,
// so a wave's reads fall into distinct banks), coefficients in FP32.
template <int RAD, int BC, bool VEC>
__global__ __launch_bounds__(k1Threads) void k_lds1d(MmaArgs p) {
    static_assert(RAD >= 1 && RAD <= k1Halo, "radius within the staged halo");
    constexpr int K = 2 * RAD + 1;
    constexpr int W = 16 + 2 * RAD;
    __shared__ __attribute__((aligned(16))) float lds[k1Words];
    if (p.edge_w && (int)blockIdx.x == p.total_items) {
        end_bands(p, reinterpret_cast<float(*)[kEdgeWin][kEdgeLanes]>(lds));
        return;
    }
    int j = 0;
    for (int t = 1; t < p.njobs; ++t) j = (int)blockIdx.x >= p.job[t].item0 ? t : j;
    const MmaJob g = p.job[j];
    const int n = g.nx;
    const int base = ((int)blockIdx.x - g.item0) * k1Block;
    const __attribute__((address_space(1))) float *x =
        (const __attribute__((address_space(1))) float *)static_cast<const float *>(g.in);
    stage_block<BC, VEC>(x, base - k1Halo, n, lds);
    float w[K];
#pragma unroll
    for (int o = 0; o < K; ++o) w[o] = p.w[o];
    __syncthreads();

    const int tid = threadIdx.x;
    // staged index of this thread's first input: c0 + 16 tid (c0 = 8 - RAD)
    constexpr int c0 = k1Halo - RAD;
    const float *src = lds + c0 + 17 * tid;
    float v[W];
#pragma unroll
    for (int i = 0; i < W; ++i) v[i] = src[i + ((c0 + i) >> 4)];
    float y[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        float acc = 0.0f;
#pragma unroll
        for (int o = 0; o < K; ++o) acc = __builtin_fmaf(w[o], v[i + o], acc);
        y[i] = acc;
    }
    const int valid = min(k1Block, n - base);
    float *out = static_cast<float *>(g.out) + base;
    const __amdgpu_buffer_rsrc_t orsrc = uniform_rsrc(out, valid * 4);
    const int bw = p.edge_w ? band_width(p) : 0;
    const int lo_end = min(bw, n) - base;
    const int hi_start = max(n - bw, min(bw, n)) - base;
    const bool plain = lo_end <= 0 && hi_start >= valid;
    const int o = 16 * tid;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int oc = o + 4 * c;
        if (VEC && plain) {
            const u4v yv = {__float_as_uint(y[4 * c]), __float_as_uint(y[4 * c + 1]), __float_as_uint(y[4 * c + 2]),
                            __float_as_uint(y[4 * c + 3])};
            __builtin_amdgcn_raw_buffer_store_b128(yv, orsrc, oc < valid ? (unsigned)oc * 4u : kOob, 0, 0);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int oi = oc + i;
                const bool keep = oi < valid && oi >= lo_end && oi < hi_start;
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(y[4 * c + i]), orsrc,
                                                      keep ? (unsigned)oi * 4u : kOob, 0, 0);
            }
        }
    }
}

template <int RAD>
hipError_t launch_lds1d(MmaArgs &a, hipStream_t s) {
    if (a.njobs < 1 || a.njobs > kMaxJobs) return hipErrorInvalidValue;
    int blocks = 0;
    bool vec = true;
    for (int j = 0; j < a.njobs; ++j) {
        MmaJob &g = a.job[j];
        if (g.nx < 1) return hipErrorInvalidValue;
        g.item0 = blocks;
        blocks += (g.nx + k1Block - 1) / k1Block;
        vec = vec && g.nx % 4 == 0 && ((uintptr_t)g.in % 16) == 0 && ((uintptr_t)g.out % 16) == 0;
    }
    a.total_items = blocks;
    if (a.edge_w && (a.edge_steps < 2 || a.edge_rad < 1 || a.edge_rad * a.edge_steps > k1Halo))
        return hipErrorInvalidValue;
    const dim3 grid(blocks + (a.edge_w ? 1 : 0)), block(k1Threads);
    if (a.periodic) {
        if (vec) hipLaunchKernelGGL((k_lds1d<RAD, kBcWrapN, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_lds1d<RAD, kBcWrapN, false>), grid, block, 0, s, a);
    } else {
        if (vec) hipLaunchKernelGGL((k_lds1d<RAD, kBcZero, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_lds1d<RAD, kBcZero, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <int RAD>
MmaLaunch pick1d(int mode, int part) {
    if (mode == kSparse) return part == kPartF16 ? &launch_mma1d<1, RAD, kSparse, kPartF16>
                                                 : &launch_mma1d<1, RAD, kSparse, kPartBF16>;
    return part == kPartF16 ? &launch_mma1d<1, RAD, kDense, kPartF16> : &launch_mma1d<1, RAD, kDense, kPartBF16>;
}

}  // namespace

MmaLaunch find_mma1d(int rad, int mode, int part) {
    switch (rad) {
        case 1: return pick1d<1>(mode, part);
        case 2: return pick1d<2>(mode, part);
        case 3: return pick1d<3>(mode, part);
        case 4: return pick1d<4>(mode, part);
        case 5: return pick1d<5>(mode, part);
        case 6: return pick1d<6>(mode, part);
        case 7: return pick1d<7>(mode, part);
        case 8: return pick1d<8>(mode, part);
        default: return nullptr;
    }
}

MmaLaunch find_lds_direct1d(int rad) {
    switch (rad) {
        case 1: return &launch_lds1d<1>;
        case 2: return &launch_lds1d<2>;
        case 3: return &launch_lds1d<3>;
        case 4: return &launch_lds1d<4>;
        case 5: return &launch_lds1d<5>;
        case 6: return &launch_lds1d<6>;
        case 7: return &launch_lds1d<7>;
        case 8: return &launch_lds1d<8>;
        default: return nullptr;
    }
}

}  // namespace ss
