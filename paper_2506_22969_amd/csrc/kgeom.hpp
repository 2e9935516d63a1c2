// Geometry shared by the host runtime (table building, launch shapes) and the
// 2-D MMA kernels.  A workgroup of 512 threads (8 waves of 64) owns a band 256
// outputs wide and 32 rows tall (a work item).  A unit is the 16 tiles one MMA
// covers along N (128 columns wide, NBH rows); the waves sit 2 across and 4
// down the item and each multiplies U units stacked vertically.
#pragma once

namespace ss {

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kBandX = 256;      // outputs per workgroup along x
constexpr int kNbCols = 2;       // units side by side across a band
constexpr int kItemRows = 32;    // rows of a work item
constexpr int kLdsBytes = 160 * 1024;

// State layouts: FP32 values, or bfloat16 hi and lo planes ([hi | lo], each
// a full grid of 16-bit values).
enum State { kStateF32 = 0, kStatePlanes = 1 };

template <int R1, int R2, int RAD, int STATE>
struct MmaGeom {
    static constexpr int MB = R1 * R2 / 16;            // 16-row M-blocks of A'
    // Tiles of a unit along x: a 128-column unit, except 16-wide tiles on
    // the planes state, whose units are 4 tiles across and 4 tile rows down
    // (with the row pitch below, the 16 tiles then start in 16 different
    // LDS banks)
    static constexpr bool SQUARE = STATE == kStatePlanes && R1 == 16;
    static constexpr int NBX = SQUARE ? 4 : 128 / R1;
    static constexpr int NBY = 16 / NBX;               // ... along y
    static constexpr int NBH = NBY * R2;               // rows of a unit
    static constexpr int UW = NBX * R1;                // columns of a unit
    static constexpr int NCOLS = kBandX / UW;          // units across a band
    static constexpr int U = kItemRows / (kWaves / NCOLS * NBH);  // units per wave
    static constexpr int WGH = kWaves / NCOLS * U * NBH;          // rows of a work item
    static_assert(WGH == kItemRows, "tile does not divide the work item");
    static constexpr int SROWS = WGH + 2 * RAD;        // slab rows
    // FP32 slab rows (floats): HL columns of left margin (>= RAD, a multiple
    // of 4 so that the interior starts 16-byte aligned), the band, RAD right
    // halo columns, padding to a multiple of 4 plus 4.
    static constexpr int HL = (RAD + 3) / 4 * 4;
    static constexpr int CPITCH = (HL + kBandX + RAD + 3) / 4 * 4 + 4;
    // Planes slab (bfloat16 elements): a hi part of SROWS rows of PB
    // elements, then a lo part of the same shape (LO elements further on).
    // Rows have an 8-element left margin and up to 8 right halo columns;
    // halo columns move in pairs (HD dwords per side and plane).  With
    // 16-wide tiles (8 dwords apart along a row, 4 per unit row) the pitch
    // makes the 4 tile rows of a unit start 2 dwords apart modulo 8:
    // R2 * PB / 2 = 2 (mod 8).  A pitch that is a multiple of 8 keeps every
    // row 16-byte aligned (LDS DMA in 16-byte pieces); otherwise rows move
    // in 4-byte pieces.
    static constexpr int HLB = 8;
    static constexpr int PB = !SQUARE ? 280 : R2 == 1 ? 276 : 274;
    static constexpr bool PLANES_X4 = PB % 8 == 0;
    static constexpr int LO = SROWS * PB;
    static constexpr int HD = (RAD + 1) / 2;
    static_assert(STATE == kStateF32 || 2 * HD <= HLB, "halo wider than the margin");
    static_assert(PB >= HLB + kBandX + 2 * HD && PB % 2 == 0, "plane row pitch");
    static_assert(!SQUARE || (R2 * PB / 2) % 8 == 2, "plane row pitch does not spread the banks");
    // with an even radius every B register's two values share one dword
    // (tile origins and pair columns are even)
    static constexpr bool PAIR_DWORD = STATE == kStatePlanes && RAD % 2 == 0;
    // per slab: elements between consecutive source rows, left margin, bytes
    static constexpr int ROW = STATE == kStateF32 ? CPITCH : PB;
    static constexpr int MARGIN = STATE == kStateF32 ? HL : HLB;
    static constexpr int SLAB_BYTES = STATE == kStateF32 ? SROWS * CPITCH * 4 : 2 * SROWS * PB * 2;
    // halo dwords of one slab, and the staging strip they land in (whole
    // 512-lane transfers)
    static constexpr int HALO_ROW = STATE == kStateF32 ? 2 * RAD : 4 * HD;
    static constexpr int NHALO = SROWS * HALO_ROW;
    static constexpr int HOPS = (NHALO + kThreads - 1) / kThreads;
    static constexpr int HSTRIP = HOPS * kThreads;
    // pipeline depth: four slabs when they fit, else three
    static constexpr int NSLAB = 4 * (SLAB_BYTES + 4 * HSTRIP) <= kLdsBytes ? 4 : 3;
    static_assert(NSLAB * (SLAB_BYTES + 4 * HSTRIP) <= kLdsBytes, "slabs exceed LDS");
};

// 3-D kernel: a work item is a column of the grid (a 256-column band of
// WGH rows) over a range of z planes; the workgroup marches through z with a
// ring of NP plane slabs in LDS, each output plane using the 2*RAD+1 input
// planes around it.  Each wave multiplies one unit (16 tiles) per plane.
// A slab row holds the band's 256 values at HL and four halo values on each
// side (whole 16-byte transfers), so RAD is at most 4.
template <int R1, int R2, int RAD>
struct Mma3Geom {
    static constexpr int MB = R1 * R2 / 16;
    static constexpr int NBX = 128 / R1;
    static constexpr int NBY = 16 / NBX;
    static constexpr int NBH = NBY * R2;
    static constexpr int WGH = kWaves / kNbCols * NBH;  // rows of a work item
    static constexpr int SROWS = WGH + 2 * RAD;
    static constexpr int HL = 4;
    static constexpr int CPITCH = (HL + kBandX + RAD + 3) / 4 * 4 + 4;
    static constexpr int PLANE_BYTES = SROWS * CPITCH * 4;
    static constexpr int NP = kLdsBytes / PLANE_BYTES < 8 ? kLdsBytes / PLANE_BYTES : 8;  // ring slots
    static_assert(RAD <= 4 && CPITCH >= HL + kBandX + 4, "slab row holds four halo values a side");
    static_assert(NP >= 2 * RAD + 2, "ring too small for the stencil depth");
};

}  // namespace ss
