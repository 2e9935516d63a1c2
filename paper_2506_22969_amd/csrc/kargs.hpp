// Kernel argument blocks and launch entry points shared by the runtime and
// the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ss {

enum Mode { kSparse = 0, kDense = 1 };
enum PartType { kPartF16 = 0, kPartBF16 = 1 };

// 2-D MMA sweep on an FP32 state split into hi+lo parts in the kernel.
struct MmaArgs {
    const float *in;
    float *out;
    int ny, nx;
    int periodic;
    float inv_sigma;
    const uint4 *a_hi;       // [MB][KC][64] A fragments (8 x 16-bit each)
    const uint4 *a_lo;
    const uint32_t *a_idx;   // [MB][KC][64] sparse index words (sparse mode)
    const int32_t *boff;     // [KC][4][VPK] gather offsets in u16 units
};

// Direct sweep: one (2r+1)^3 box (r = 0 on missing axes).
struct DirectArgs {
    const void *in;
    void *out;
    int nz, ny, nx;
    int rz, ry, rx;
    int periodic;
    const void *w;           // coefficients, same type as the state
};

// Key of an instantiated 2-D MMA kernel.
struct MmaKey {
    int r1, r2, kc, rad, mode, part;
};

// Returns nullptr when no kernel is instantiated for the key.
using MmaLaunch = hipError_t (*)(const MmaArgs &, hipStream_t);
MmaLaunch find_mma2d(const MmaKey &key);
bool mma2d_geometry(const MmaKey &key, int *wgh, int *pitch, int *F, int *S);

hipError_t launch_direct(const DirectArgs &a, int is_f64, hipStream_t s);

}  // namespace ss
