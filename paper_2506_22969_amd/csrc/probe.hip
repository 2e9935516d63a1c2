// Matrix-core throughput probe: the measured peak that the sweeps' matrix
// utilisation is reported against (the spec sheet's figure is not measured
// on the part at hand).  Every wave runs chains of independent products on
// register operands only (no memory traffic besides one store of the
// accumulators at the end, which keeps the products live).
#include <hip/hip_runtime.h>

#include "../../include/sparstencil.h"
#include "kargs.hpp"

namespace ss {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h16 __attribute__((ext_vector_type(16)));

constexpr int kChains = 8;        // independent accumulators per wave

template <bool SPARSE>
__global__ __launch_bounds__(256) void k_mma_peak(long long iters, float *out) {
    const int lane = threadIdx.x & 63;
    h8 a;
    h16 b;
    for (int e = 0; e < 8; ++e) a[e] = (_Float16)(0.001f * (lane + e));
    for (int e = 0; e < 16; ++e) b[e] = (_Float16)(0.001f * (lane - e));
    f4 acc[kChains];
    for (int c = 0; c < kChains; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
    const int idx = 0x44444444 ^ lane;   // any 2-bit positions
    for (long long i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (SPARSE)
                acc[c] = __builtin_amdgcn_smfmac_f32_16x16x64_f16(a, b, acc[c], idx, 0, 0);
            else
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b.lo, acc[c], 0, 0, 0);
        }
    }
    f4 s = acc[0];
    for (int c = 1; c < kChains; ++c) s += acc[c];
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    reinterpret_cast<f4 *>(out)[t] = s;
}

}  // namespace
}  // namespace ss

extern "C" ss_status sparstencil_probe_mma_peak(int32_t engine, int64_t iters, int32_t workgroups, float *out,
                                                double *flops, void *stream) {
    if (!out || !flops || iters < 1 || workgroups < 1 || workgroups > (1 << 20) ||
        (engine != SS_ENGINE_SMFMAC && engine != SS_ENGINE_MFMA))
        return SS_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool sparse = engine == SS_ENGINE_SMFMAC;
    if (sparse)
        hipLaunchKernelGGL(ss::k_mma_peak<true>, dim3(workgroups), dim3(256), 0, s, (long long)iters, out);
    else
        hipLaunchKernelGGL(ss::k_mma_peak<false>, dim3(workgroups), dim3(256), 0, s, (long long)iters, out);
    if (hipGetLastError() != hipSuccess) return SS_E_DEVICE;
    // dense-equivalent flops: 16 x 16 x K multiply-adds per product, K = 64
    // (sparse, half of them structural zeros) or 32 (dense)
    const double per = 2.0 * 16 * 16 * (sparse ? 64 : 32);
    *flops = per * (double)iters * ss::kChains * (double)workgroups * 4.0;
    return SS_OK;
}
