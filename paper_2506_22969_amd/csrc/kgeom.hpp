// Geometry shared by the host runtime (table building, launch shapes) and the
// 2-D / 3-D MMA kernels.  A workgroup of 256 threads (4 waves of 64) owns a
// band 128 outputs wide; an N-block is the 16 tiles one MMA covers along N.
#pragma once

namespace ss {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kBandX = 128;      // outputs per workgroup along x
constexpr int kNbw = 2;          // N-blocks per wave

template <int R1, int R2, int RAD>
struct MmaGeom {
    static constexpr int MB = R1 * R2 / 16;          // 16-row M-blocks of A'
    static constexpr int NBX = kBandX / R1;          // tiles of an N-block along x
    static constexpr int NBY = 16 / NBX;             // ... along y
    static constexpr int NBH = NBY * R2;             // rows of an N-block
    static constexpr int WGH = kWaves * kNbw * NBH;  // rows of a workgroup
    static constexpr int SROWS = WGH + 2 * RAD;      // slab rows
    static constexpr int CPS = (kBandX + 2 * RAD + 1) / 2;  // column pairs per slab row
    // Column pairs are interleaved by F = R1/2 (pairs per tile): logical pair
    // cp lives at physical slot (cp % F) * S + cp / F, so the 16 lanes of an
    // N-block, whose patches start F pairs apart, read adjacent slots.
    static constexpr int F = R1 / 2;
    static constexpr int S = (CPS + F - 1) / F;
    static constexpr int PITCH = 4 * F * S + 4;      // u16 per slab row (hi,hi,lo,lo per pair)
    static constexpr int SLAB_U16 = SROWS * PITCH;
};

__host__ __device__ constexpr inline int pair_slot(int cp, int F, int S) { return (cp % F) * S + cp / F; }

}  // namespace ss
