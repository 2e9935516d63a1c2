// Geometry shared by the host runtime (table building, launch shapes) and the
// 2-D MMA kernels.  A workgroup of 512 threads (8 waves of 64) owns a band 256
// outputs wide and 32 rows tall (a work item).  A unit is the 16 tiles one MMA
// covers along N (UW columns wide, NBH rows); the waves sit side by side
// across the item (NCOLS unit columns) and down it, and each multiplies U
// units stacked vertically.
#pragma once

namespace ss {

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kBandX = 256;      // outputs per workgroup along x
constexpr int kNbCols = 2;       // units side by side across a band
constexpr int kItemRows = 32;    // rows of a work item
constexpr int kLdsBytes = 160 * 1024;

// State layouts: FP32 values, bfloat16 hi and lo planes ([hi | lo], each a
// full grid of 16-bit values), plain binary16 values, or bfloat16 hi, mid
// and lo planes ([hi | mid | lo]).
enum State { kStateF32 = 0, kStatePlanes = 1, kStateF16 = 2, kStatePlanes3 = 3 };

template <int R1, int R2, int RAD, int STATE>
struct MmaGeom {
    static constexpr int MB = R1 * R2 / 16;            // 16-row M-blocks of A'
    // Tiles of a unit along x: a 128-column unit, except 16-wide tiles on
    // the planes state, whose units are 2 tiles across and 8 tile rows down
    // (with the row pitch below, the 16 tiles then start in 16 different
    // pairs of LDS banks)
    static constexpr bool TALL = STATE == kStatePlanes && R1 == 16;
    static constexpr int NBX = TALL ? 2 : 128 / R1;
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
    // Planes slab: rows of RBD dwords in which hi and lo pairs alternate:
    // dword 2m + p holds values 2m and 2m+1 of plane p (0 hi, 1 lo), counted
    // from HLB values left of the band, so that one 8-byte read returns a B
    // register's hi and lo parts.  A row holds HLB = 8 values of left
    // margin, the band and 8 values on the right (272 dwords; RAD <= 8), all
    // moved by the row's own 4-byte transfers.  16-wide tiles are 16 dwords
    // apart along a row; the pitch puts the 8 tile rows of a unit 2 dwords
    // apart modulo 32: R2 * RBD = 2 (mod 32).
    static constexpr int HLB = 8;
    static constexpr int RBD = TALL && R2 == 1 ? 290 : 273;
    static_assert(STATE == kStateF32 || (RAD <= HLB && RBD >= 2 * HLB + kBandX),
                  "planes slab row");
    static_assert(!TALL || (R2 * RBD) % 32 == 2, "plane row pitch does not spread the banks");
    // with an even radius every B register's two values share one dword of
    // each plane (tile origins and pair columns are even)
    static constexpr bool PAIR_DWORD = STATE == kStatePlanes && RAD % 2 == 0;
    // per slab: distance between consecutive source rows (FP32 values;
    // planes bytes), left margin (values), bytes
    static constexpr int ROW = STATE == kStateF32 ? CPITCH : 4 * RBD;
    static constexpr int MARGIN = STATE == kStateF32 ? HL : HLB;
    static constexpr int SLAB_BYTES = STATE == kStateF32 ? SROWS * CPITCH * 4 : SROWS * RBD * 4;
    // FP32 halo dwords of one slab, and the staging strip they land in
    // (whole 512-lane transfers); the planes rows carry their own halo
    static constexpr int HALO_ROW = STATE == kStateF32 ? 2 * RAD : 0;
    static constexpr int NHALO = SROWS * HALO_ROW;
    static constexpr int HOPS = (NHALO + kThreads - 1) / kThreads;
    static constexpr int HSTRIP = HOPS * kThreads;
    // pipeline depth: four slabs when they fit, else three
    static constexpr int NSLAB = 4 * (SLAB_BYTES + 4 * HSTRIP) <= kLdsBytes ? 4 : 3;
    static_assert(NSLAB * (SLAB_BYTES + 4 * HSTRIP) <= kLdsBytes, "slabs exceed LDS");
};

// Staged-and-converted slabs of the 2-D matrix kernels on an FP32 or a
// binary16 state.  A work item's rows land by LDS DMA in a staging slab as
// stored: SPITCH values per row, the 256-value band between one 16-byte piece
// of halo on either side (so RAD <= CH), for a bfloat16 hi/lo planes state
// the hi row and then the lo row.  One pass then writes every horizontal
// pair of values (columns P0 + 2j and P0 + 2j + 1 of the staging row, P0
// being the first column any tile reads) in the form a B register takes: an
// FP32 pair as its packed hi word and packed lo word, a planes pair as its
// hi-plane word and lo-plane word (PW = 2 dwords), a binary16 pair as one
// word (PW = 1).  Pair j of a converted row
// sits at dword pos(j) = PW * (j + j / PADG): a gap of PW dwords after every
// PADG pairs, so that the 16 tiles of a unit start in 16 different LDS banks
// (pairs of banks for PW = 2); the row pitch ROWC is chosen for the same
// purpose when a unit spans two tile rows.  Tile origins are whole multiples
// of PADG pairs, so pos(origin + j) = pos(origin) + pos(j): one gather
// offset table serves every tile.
template <int R1, int R2, int RAD, int STATE>
struct ConvGeom {
    using G = MmaGeom<R1, R2, RAD, kStateF32>;         // unit arrangement
    static constexpr int EB = STATE == kStateF32 ? 4 : 2;    // bytes per stored value
    static constexpr int NPL = STATE == kStatePlanes3 ? 3 : STATE == kStatePlanes ? 2 : 1;   // stored planes
    static constexpr int CH = 16 / EB;                       // values per 16-byte piece
    static constexpr int SPITCH = kBandX + 2 * CH;           // staged values per row and plane
    static constexpr int PIECES = SPITCH / CH;               // 16-byte pieces per row and plane
    static constexpr int SROWS = G::SROWS;
    // a staging row holds the row of every plane, one after the other
    static constexpr int NPIECE = SROWS * NPL * PIECES;
    static constexpr int STAGE_BYTES = SROWS * NPL * SPITCH * EB;
    static constexpr int P0 = CH - RAD;
    static constexpr int NPAIR = kBandX / 2 + RAD;           // pairs per row
    // dwords per converted pair: one word per part (hi and lo; hi, mid and lo)
    static constexpr int PW = STATE == kStateF16 ? 1 : STATE == kStatePlanes3 ? 3 : 2;
    static constexpr int PADG = R1 == 8 ? 4 : 8;
    static constexpr int pos(int j) { return PW * (j + j / PADG); }
    // first dword of each of the 16 tiles of a unit, modulo 32 banks, all
    // different (PW = 2: all even and different; PW = 3 cannot avoid every
    // conflict of its 48 dwords, its first dwords differ)
    static constexpr bool banks_ok(int rowc) {
        int seen[32] = {};
        for (int n = 0; n < 16; ++n) {
            const int b = ((n / G::NBX) * R2 * rowc + pos((n % G::NBX) * R1 / 2)) % 32;
            if ((PW == 2 && b % 2 != 0) || seen[b]) return false;
            seen[b] = 1;
        }
        return true;
    }
    static constexpr int pick_rowc() {
        const int lo = (pos(NPAIR - 1) + PW + 1) / 2 * 2;      // even: 8-byte aligned pairs
        for (int r = lo; r < lo + 64; r += 2)
            if (banks_ok(r)) return r;
        return lo;
    }
    static constexpr int ROWC = pick_rowc();
    static constexpr int CONV_BYTES = SROWS * ROWC * 4;
    // a staging slab is followed by room for the transfers that round its
    // pieces (or, FP32 rows not 16-byte aligned, values) up to whole
    // 512-lane rounds, so that every lane of every round is active
    static constexpr int ROUND_VEC = (NPIECE + 511) / 512 * 512 * 16;
    static constexpr int ROUND_ELEM = STATE == kStateF32 ? (SROWS * SPITCH + 511) / 512 * 512 * 4 : 0;
    static constexpr int STAGE_ALLOC = ROUND_VEC > ROUND_ELEM ? ROUND_VEC : ROUND_ELEM;
    // staging slabs: two, or one when two do not fit beside the converted
    // slab (three planes of a wide stencil)
    static constexpr int NSLAB = CONV_BYTES + 2 * STAGE_ALLOC <= kLdsBytes ? 2 : 1;
    static constexpr int LDS_BYTES = CONV_BYTES + NSLAB * STAGE_ALLOC;
    static_assert(RAD <= CH && P0 >= 0, "halo wider than one 16-byte piece");
    static_assert(R1 % (2 * PADG) == 0 && (G::UW / 2) % PADG == 0, "tile origins off the gap grid");
    static_assert(banks_ok(ROWC), "no row pitch spreads the tiles over the banks");
    static_assert(LDS_BYTES <= kLdsBytes, "slabs exceed LDS");
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

// Converted plane of the 3-D matrix kernels: the pairs of a staged FP32
// plane from column P0 = HL - RAD on (the first column any tile reads), each
// as its packed hi word and packed lo word (PW = 2 dwords), pair j of a row
// at dword pos(j) = PW * (j + j / PADG) and rows ROWC dwords apart -- the
// 2-D kernels' converted layout, which starts the 16 tiles of a unit in 16
// different bank pairs.  The ring of staged planes gives up the room.
template <int R1, int R2, int RAD>
struct Conv3Geom {
    using G = Mma3Geom<R1, R2, RAD>;
    static constexpr int P0 = G::HL - RAD;
    static constexpr int NPAIR = kBandX / 2 + RAD;
    static constexpr int PW = 2;
    static constexpr int PADG = R1 == 8 ? 4 : 8;
    static constexpr int pos(int j) { return PW * (j + j / PADG); }
    static constexpr bool banks_ok(int rowc) {
        int seen[32] = {};
        for (int n = 0; n < 16; ++n) {
            const int b = ((n / G::NBX) * R2 * rowc + pos((n % G::NBX) * R1 / 2)) % 32;
            if (b % 2 != 0 || seen[b]) return false;
            seen[b] = 1;
        }
        return true;
    }
    static constexpr int pick_rowc() {
        const int lo = (pos(NPAIR - 1) + PW + 1) / 2 * 2;
        for (int r = lo; r < lo + 64; r += 2)
            if (banks_ok(r)) return r;
        return lo;
    }
    static constexpr int ROWC = pick_rowc();
    static constexpr int CONV_BYTES = G::SROWS * ROWC * 4;
    static constexpr int NPF = (kLdsBytes - CONV_BYTES) / G::PLANE_BYTES;
    static constexpr int NP = NPF < 8 ? NPF : 8;                       // ring slots
    static_assert(P0 >= 0 && (R1 / 2) % PADG == 0 && (128 / 2) % PADG == 0, "tile origins off the gap grid");
    static_assert(banks_ok(ROWC), "no row pitch spreads the tiles over the banks");
    static_assert(NP >= 2 * RAD + 2, "ring too small for the stencil depth");
};

}  // namespace ss
