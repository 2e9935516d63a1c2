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
    const void *in;
    void *out;
    int ny, nx;
    int item0;
    int nz, zc;              // 3-D: planes, and planes per work item
};

// 2-D MMA sweep: FP32 state split into hi+lo parts in the kernel, or a state
// of bfloat16 hi and lo planes.
struct MmaArgs {
    int njobs;
    int total_items;         // work items over all jobs
    int nxcd;                // XCDs the launch's workgroups are dealt over
    MmaJob job[kMaxJobs];
    int periodic;
    float inv_sigma;
    const uint4 *a_hi;       // [MB][KC][64] A fragments (8 x 16-bit each)
    const uint4 *a_lo;
    const uint4 *a_mid;      // three-part states: the coefficients' mid parts
    const uint32_t *a_idx;   // [MB][KC][64] sparse index words (sparse mode)
    const int32_t *boff;     // [KC][4][VPK] gather offsets in bytes
    const void *zeros;       // 1 KiB of zeros (loads outside a zero-halo grid)
    const float *w;          // (2r+1)^2 coefficients (direct LDS kernel only)
    // fused zero-halo sweeps: the unfused coefficients (FP64 for the 1-D
    // kernels, FP32 for the 2-D ones), radius and S; the launch then also
    // recomputes the points within r(S-1) of the edges (edge_steps < 2: no
    // band)
    const double *edge_w;
    const float *edge_w32;
    int edge_rad, edge_steps;
};

struct DirectJob {
    const void *in;
    void *out;
    int nz, ny, nx;
    int block0;
};

// Edge correction of a fused launch of S sweeps on a 2-D zero-halo grid:
// the points within r(S-1) of an edge get the exact S-sweep value.
struct EdgeJob {
    const float *in;   // state the fused launch read
    float *out;        // the fused launch's output (band points overwritten)
    int ny, nx;
    int point0;        // first band point of this grid in the launch
};
struct EdgeArgs {
    int njobs;
    int total;
    EdgeJob job[kMaxJobs];
    int rad;
    int steps;         // S: 2, or 3 for radius 1
    const double *w;   // the unfused (2r+1)^2 coefficients
};
hipError_t launch_edge2d(EdgeArgs &a, hipStream_t s);

// Direct sweep: one (2r+1)^3 box (r = 0 on missing axes), radius up to
// kDirectMaxRad.
constexpr int kDirectMaxRad = 6;
struct DirectArgs {
    int njobs;
    int total_blocks;
    DirectJob job[kMaxJobs];
    int rz, ry, rx;
    int periodic;
    const void *w;           // coefficients (FP64 for an FP64 state, else FP32)
    int steps;               // sweeps per launch of the temporal-block kernel
};

// Key of an instantiated 2-D MMA kernel.
struct MmaKey {
    int r1, r2, kc, rad, mode, part, state;
};

// Returns nullptr when no kernel is instantiated for the key.  The launch
// fills total_items and the jobs' item0 from their grid sizes.
using MmaLaunch = hipError_t (*)(MmaArgs &, hipStream_t);
MmaLaunch find_mma2d(const MmaKey &key);
// Rows of a work item and the gather row pitch (FP32 slab: values; planes:
// bytes; converted slab: dwords), and for a converted slab the dwords per
// pair and pairs between row gaps (pw = 0 otherwise).
bool mma2d_geometry(const MmaKey &key, int *wgh, int *row, int *pw, int *padg);
// Instantiated keys with the given radius, mode, part and state (at most max).
int mma2d_keys(int rad, int mode, int part, int state, MmaKey *out, int max);

// State types of the direct engine: FP32, FP64 (coefficients of the same
// type), bfloat16 hi and lo planes (FP32 coefficients and arithmetic).
enum DirectKind { kDirectF32 = 0, kDirectF64 = 1, kDirectPlanes = 2 };

// 3-D MMA kernels (FP32 state), same conventions; the launch also fills the
// jobs' z-chunk depth zc.
MmaLaunch find_mma3d(const MmaKey &key);
// Rows of a work item and the converted plane's row pitch (dwords), dwords
// per pair and pairs between row gaps.
bool mma3d_geometry(const MmaKey &key, int *wgh, int *row, int *pw, int *padg);
int mma3d_keys(int rad, int mode, int part, MmaKey *out, int max);

// Direct 2-D sweep from the same LDS-DMA slab pipeline (FP32 state or
// bfloat16 planes); nullptr when no kernel exists for the radius.
MmaLaunch find_lds_direct2d(int rad, int state);

// Direct 3-D sweep (FP32 state) from the same z-march pipeline as the 3-D
// matrix kernels; nullptr when no kernel exists for the radius.
MmaLaunch find_lds_direct3d(int rad);

// 1-D MMA sweep (FP32 state, tile of 16 outputs, one K chunk) for radius
// 1..8; nullptr beyond.  The launch fills total_items and the jobs' item0.
MmaLaunch find_mma1d(int rad, int mode, int part);
// Direct 1-D sweep (FP32 state) from the same staging, radius 1..8,
// coefficients in MmaArgs::w; nullptr beyond.
MmaLaunch find_lds_direct1d(int rad);

// Dense FP64 MMA sweep (tile 8 x 4, FP64 state and coefficients): the
// launch for radius `rad` and KC chunks of 4, and its slab row pitch.
MmaLaunch find_mma2d_f64(int rad, int kc);
int mma2d_f64_pitch(int rad);

// Fills total_blocks and the jobs' block0 from their grid sizes.
hipError_t launch_direct(DirectArgs &a, int kind, hipStream_t s);

// Several sweeps of one small 2-D FP64 grid in one launch (temporal
// blocking, a.steps sweeps with a.steps * radius <= kTbHalo, radius <= 4).
constexpr int kTbHalo = 16;
hipError_t launch_direct_tb(DirectArgs &a, hipStream_t s);

}  // namespace ss
