// Geometry shared by the host runtime (table building, launch shapes) and the
// 2-D MMA kernels.  A workgroup of 512 threads (8 waves of 64) owns a band 256
// outputs wide; an N-block is the 16 tiles one MMA covers along N (128
// columns wide), and each wave multiplies one N-block of every work item.
#pragma once

namespace ss {

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kBandX = 256;      // outputs per workgroup along x
constexpr int kNbCols = 2;       // N-blocks side by side across a band
constexpr int kSlabs = 4;        // LDS slabs in the load pipeline

template <int R1, int R2, int RAD>
struct MmaGeom {
    static constexpr int MB = R1 * R2 / 16;            // 16-row M-blocks of A'
    static constexpr int NBX = 128 / R1;               // tiles of an N-block along x
    static constexpr int NBY = 16 / NBX;               // ... along y
    static constexpr int NBH = NBY * R2;               // rows of an N-block
    static constexpr int WGH = kWaves / kNbCols * NBH;  // rows of a work item
    static constexpr int SROWS = WGH + 2 * RAD;        // slab rows
    // FP32 slab rows: HL columns of left margin (>= RAD, a multiple of 4, so
    // that the interior columns start 16-byte aligned), the band, RAD right
    // halo columns, padding to a multiple of 4 plus 4.
    static constexpr int HL = (RAD + 3) / 4 * 4;
    static constexpr int CPITCH = (HL + kBandX + RAD + 3) / 4 * 4 + 4;  // floats per slab row
    static constexpr int SLAB_F = SROWS * CPITCH;                       // floats per slab
};

}  // namespace ss
