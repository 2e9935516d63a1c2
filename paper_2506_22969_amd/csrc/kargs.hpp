// Kernel argument blocks and launch entry points shared by the runtime and
// the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ss {

enum Mode { kSparse = 0, kDense = 1 };
enum PartType { kPartF16 = 0, kPartBF16 = 1 };

// Grids one launch sweeps (several jobs of the same plan tables can share a
// launch).  item0 / block0: index of the job's first work item / block.
constexpr int kMaxJobs = 16;

struct MmaJob {
    const float *in;
    float *out;
    int ny, nx;
    int item0;
};

// 2-D MMA sweep on an FP32 state split into hi+lo parts in the kernel.
struct MmaArgs {
    int njobs;
    int total_items;         // work items over all jobs
    int nxcd;                // XCDs the launch's workgroups are dealt over
    MmaJob job[kMaxJobs];
    int periodic;
    float inv_sigma;
    const uint4 *a_hi;       // [MB][KC][64] A fragments (8 x 16-bit each)
    const uint4 *a_lo;
    const uint32_t *a_idx;   // [MB][KC][64] sparse index words (sparse mode)
    const int32_t *boff;     // [KC][4][VPK] gather offsets in floats
    const float *zeros;      // 1 KiB of zeros (loads outside a zero-halo grid)
};

struct DirectJob {
    const void *in;
    void *out;
    int nz, ny, nx;
    int block0;
};

// Direct sweep: one (2r+1)^3 box (r = 0 on missing axes).
struct DirectArgs {
    int njobs;
    int total_blocks;
    DirectJob job[kMaxJobs];
    int rz, ry, rx;
    int periodic;
    const void *w;           // coefficients, same type as the state
};

// Key of an instantiated 2-D MMA kernel.
struct MmaKey {
    int r1, r2, kc, rad, mode, part;
};

// Returns nullptr when no kernel is instantiated for the key.  The launch
// fills total_items and the jobs' item0 from their grid sizes.
using MmaLaunch = hipError_t (*)(MmaArgs &, hipStream_t);
MmaLaunch find_mma2d(const MmaKey &key);
bool mma2d_geometry(const MmaKey &key, int *wgh, int *cpitch);

// Fills total_blocks and the jobs' block0 from their grid sizes.
hipError_t launch_direct(DirectArgs &a, int is_f64, hipStream_t s);

}  // namespace ss
