// Direct 2-D stencil sweep on the vector ALUs, fed by the same persistent
// LDS-DMA slab pipeline as the matrix-core kernels (the same-box baseline
// without the matrix product): each thread computes a column of 16 outputs
// of a 256 x 32 work item, reading every slab value it needs once into
// registers and applying the (2r+1)^2 coefficients (scalar operands) with
// FP32 fused multiply-adds.
#include <hip/hip_runtime.h>

#include "mma2d_impl.hpp"

namespace ss {

namespace {

constexpr int kRowsPerThread = kItemRows / (kThreads / kBandX);  // 16

template <int RAD, int STATE, bool VEC>
struct DPipe {
    using G = MmaGeom<8, 8, RAD, STATE>;
    using P = Pipe<8, 8, RAD, STATE, VEC>;
    static constexpr int D = P::D;                                        // loads per wave per item
    static constexpr int M = kRowsPerThread * (STATE == kStatePlanes ? 2 : 1);  // stores per wave per item
    template <int S>
    static constexpr int W = (G::NSLAB - 2) * D + (S < G::NSLAB - 1 ? S : G::NSLAB - 1) * M;
};

template <int RAD, int STATE, bool VEC>
__device__ inline void direct_item(const MmaJob &g, const float *wl, const char *slab, int X0, int Y0) {
    using G = MmaGeom<8, 8, RAD, STATE>;
    constexpr int K = 2 * RAD + 1;
    const int c = threadIdx.x % kBandX;
    const int y0 = (threadIdx.x / kBandX) * kRowsPerThread;  // first output row of this thread in the item
    X0 = __builtin_amdgcn_readfirstlane(X0);
    Y0 = __builtin_amdgcn_readfirstlane(Y0);
    float acc[kRowsPerThread];
#pragma unroll
    for (int y = 0; y < kRowsPerThread; ++y) acc[y] = 0.f;
    // coefficients come from an LDS copy (one broadcast read each, where it
    // is used): the empty asm stops the compiler from hoisting all (2r+1)^2
    // of them out of the item loop into registers
    int wbase = 0;
    asm volatile("" : "+v"(wbase));
    const float *w = wl + wbase;
    // slab row r holds grid row Y0 - RAD + r: output row y reads slab rows
    // y .. y + 2*RAD.  One slab column (16 + 2*RAD values) at a time, with
    // that column's 2*RAD+1 coefficients
#pragma unroll
    for (int dx = 0; dx < K; ++dx) {
        // the empty asm statements pin the column's reads after the previous
        // column's products and its products before the next column's reads,
        // so that one column is live at a time (the scheduler would otherwise
        // hoist every column's reads and run out of registers)
        int col = G::MARGIN - RAD + c + dx;
        asm volatile("" : "+v"(col));
        float v[kRowsPerThread + 2 * RAD];
#pragma unroll
        for (int ry = 0; ry < kRowsPerThread + 2 * RAD; ++ry) {
            // planes slabs hold FP32 values by now (planes_to_f32)
            v[ry] = reinterpret_cast<const float *>(slab)[(y0 + ry) * (STATE == kStatePlanes ? G::RBD : G::CPITCH) + col];
        }
#pragma unroll
        for (int dy = 0; dy < K; ++dy) {
            const float wc = w[dy * K + dx];
#pragma unroll
            for (int y = 0; y < kRowsPerThread; ++y) acc[y] = fmaf(wc, v[y + dy], acc[y]);
        }
#pragma unroll
        for (int y = 0; y < kRowsPerThread; ++y) asm volatile("" : "+v"(acc[y]));
    }
    const int rows_left = min(G::WGH, g.ny - Y0);
    const int gx = X0 + c;
    if constexpr (STATE == kStatePlanes) {
        unsigned short *out = static_cast<unsigned short *>(g.out);
        const size_t plane = (size_t)g.ny * g.nx;
        const __amdgpu_buffer_rsrc_t rh = uniform_rsrc(out + (size_t)Y0 * g.nx, rows_left * g.nx * 2);
        const __amdgpu_buffer_rsrc_t rl = uniform_rsrc(out + plane + (size_t)Y0 * g.nx, rows_left * g.nx * 2);
#pragma unroll
        for (int y = 0; y < kRowsPerThread; ++y) {
            const __bf16 hb = (__bf16)acc[y];
            const __bf16 lb = (__bf16)(acc[y] - (float)hb);
            const unsigned o = y0 + y < rows_left && gx < g.nx ? (unsigned)((y0 + y) * g.nx + gx) * 2u : kOob;
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, hb), rh, o, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, lb), rl, o, 0, 0);
        }
    } else {
        float *out = static_cast<float *>(g.out);
        const __amdgpu_buffer_rsrc_t r = uniform_rsrc(out + (size_t)Y0 * g.nx, rows_left * g.nx * 4);
#pragma unroll
        for (int y = 0; y < kRowsPerThread; ++y) {
            const unsigned o = y0 + y < rows_left && gx < g.nx ? (unsigned)((y0 + y) * g.nx + gx) * 4u : kOob;
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[y]), r, o, 0, 0);
        }
    }
}

// Planes slab rows hold hi and lo dword pairs: (hi, lo) of values 2m, 2m+1
// at dwords 2m, 2m+1.  Replacing each pair by the two FP32 values hi + lo
// (exact in FP32) leaves value column c at dword c: an FP32 slab of row pitch
// RBD, which the direct computation reads once per use.
template <int RAD>
__device__ inline void planes_to_f32(char *slab) {
    using G = MmaGeom<8, 8, RAD, kStatePlanes>;
    constexpr int PAIRS = (2 * G::HLB + kBandX) / 2;   // dword pairs a row holds
    for (int e = threadIdx.x; e < G::SROWS * PAIRS; e += kThreads) {
        unsigned *w = reinterpret_cast<unsigned *>(slab) + (e / PAIRS) * G::RBD + 2 * (e % PAIRS);
        const unsigned hi = w[0], lo = w[1];
        w[0] = __float_as_uint(__uint_as_float(hi << 16) + __uint_as_float(lo << 16));
        w[1] = __float_as_uint(__uint_as_float(hi & 0xffff0000u) + __uint_as_float(lo & 0xffff0000u));
    }
}

template <int RAD, int STATE, bool VEC, int BC>
__global__ __launch_bounds__(kThreads, 1) void k_lds2d(MmaArgs p) {
    using G = MmaGeom<8, 8, RAD, STATE>;
    using DP = DPipe<RAD, STATE, VEC>;
    constexpr int NS = G::NSLAB;
    __shared__ __attribute__((aligned(16))) char lds[NS * (G::SLAB_BYTES + 4 * G::HSTRIP)];
    __shared__ float wl[(2 * RAD + 1) * (2 * RAD + 1)];
    auto slab = [&](int i) { return lds + i * G::SLAB_BYTES; };
    auto strip = [&](int i) { return reinterpret_cast<unsigned *>(lds + NS * G::SLAB_BYTES) + i * G::HSTRIP; };
    // XCD-aware contiguous item ranges, as in the matrix-core kernels
    const int nxcd = p.nxcd;
    const int nwg = gridDim.x;
    const int xcd = blockIdx.x % nxcd;
    const int stride = nwg / nxcd + (xcd < nwg % nxcd ? 1 : 0);
    const int before = xcd * (nwg / nxcd) + min(xcd, nwg % nxcd);
    const int range_begin = (int)((long long)p.total_items * before / nwg);
    const int total = (int)((long long)p.total_items * (before + stride) / nwg);
    const int first = range_begin + blockIdx.x / nxcd;
    if (first >= total) return;
    for (int i = threadIdx.x; i < (2 * RAD + 1) * (2 * RAD + 1); i += kThreads) wl[i] = p.w[i];
    // the copy's global loads are the only VMEM loads the compiler tracks
    wait_vmcnt<0>();
    __syncthreads();
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
        issue_item<8, 8, RAD, STATE, VEC, BC>(p.zeros, p.job[j], slab(s % NS), strip(s % NS), X0, Y0);
    };
#pragma unroll
    for (int s = 0; s < NS - 1; ++s) issue(s);
#pragma unroll 1
    for (int s = 0;; ++s) {
        switch (s) {
            case 0: wait_vmcnt<DP::template W<0>>(); break;
            case 1: wait_vmcnt<DP::template W<1>>(); break;
            case 2: wait_vmcnt<DP::template W<2>>(); break;
            default: wait_vmcnt<DP::template W<3>>(); break;
        }
        const int cur = s % NS;
        __builtin_amdgcn_s_barrier();
        if constexpr (G::NHALO > 0) {
            put_halo<8, 8, RAD, STATE>(slab(cur), strip(cur));
            __builtin_amdgcn_s_waitcnt(0xC07F);
            __builtin_amdgcn_s_barrier();
        }
        if constexpr (STATE == kStatePlanes) {
            planes_to_f32<RAD>(slab(cur));
            __builtin_amdgcn_s_waitcnt(0xC07F);      // lgkmcnt(0): converted values written
            __builtin_amdgcn_s_barrier();
        }
        issue(s + NS - 1);
        int j, X0, Y0;
        locate(item(s), j, X0, Y0);
        direct_item<RAD, STATE, VEC>(p.job[j], wl, slab(cur), X0, Y0);
        if (first + (s + 1) * stride >= total) break;
    }
    wait_vmcnt<0>();
}

template <int RAD, int STATE, bool VEC, int BC>
hipError_t launch_lds_bc(const MmaArgs &a, hipStream_t s) {
    int cus = 0, xcds = 0;
    if (const hipError_t e = device_shape(&cus, &xcds); e != hipSuccess) return e;
    MmaArgs b = a;
    b.nxcd = xcds;
    const int g = a.total_items < cus ? a.total_items : cus;
    hipLaunchKernelGGL((k_lds2d<RAD, STATE, VEC, BC>), dim3(g), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

template <int RAD, int STATE>
hipError_t launch_lds2d(MmaArgs &a, hipStream_t s) {
    using G = MmaGeom<8, 8, RAD, STATE>;
    if (a.njobs < 1 || a.njobs > kMaxJobs) return hipErrorInvalidValue;
    int items = 0;
    bool vec = true, wrap1 = true;
    for (int j = 0; j < a.njobs; ++j) {
        const MmaJob &g = a.job[j];
        a.job[j].item0 = items;
        items += ((g.nx + kBandX - 1) / kBandX) * ((g.ny + G::WGH - 1) / G::WGH);
        vec = vec && (g.nx % (STATE == kStatePlanes ? 8 : 4)) == 0;
        wrap1 = wrap1 && g.ny >= G::SROWS &&
                g.nx >= kBandX + (STATE == kStatePlanes ? 2 * G::HLB : 2 * RAD + 2);
    }
    a.total_items = items;
    if (items == 0) return hipSuccess;
    if constexpr (STATE == kStatePlanes) {
        if (!vec) return hipErrorInvalidValue;
        if (!a.periodic) return launch_lds_bc<RAD, STATE, true, kBcZero>(a, s);
        if (wrap1) return launch_lds_bc<RAD, STATE, true, kBcWrap1>(a, s);
        return launch_lds_bc<RAD, STATE, true, kBcWrapN>(a, s);
    } else {
        if (vec) {
            if (!a.periodic) return launch_lds_bc<RAD, STATE, true, kBcZero>(a, s);
            if (wrap1) return launch_lds_bc<RAD, STATE, true, kBcWrap1>(a, s);
            return launch_lds_bc<RAD, STATE, true, kBcWrapN>(a, s);
        }
        if (!a.periodic) return launch_lds_bc<RAD, STATE, false, kBcZero>(a, s);
        if (wrap1) return launch_lds_bc<RAD, STATE, false, kBcWrap1>(a, s);
        return launch_lds_bc<RAD, STATE, false, kBcWrapN>(a, s);
    }
}

}  // namespace

// Radii 1, 2, 3 and 6 (two fused radius-3 sweeps), FP32 state and planes.
MmaLaunch find_lds_direct2d(int rad, int state) {
    if (state == kStateF32) {
        switch (rad) {
            case 1: return &launch_lds2d<1, kStateF32>;
            case 2: return &launch_lds2d<2, kStateF32>;
            case 3: return &launch_lds2d<3, kStateF32>;
            case 6: return &launch_lds2d<6, kStateF32>;
        }
    } else {
        switch (rad) {
            case 1: return &launch_lds2d<1, kStatePlanes>;
            case 2: return &launch_lds2d<2, kStatePlanes>;
            case 3: return &launch_lds2d<3, kStatePlanes>;
            case 6: return &launch_lds2d<6, kStatePlanes>;
        }
    }
    return nullptr;
}

}  // namespace ss
