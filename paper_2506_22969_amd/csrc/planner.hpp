// Host-side planning: layout morphing, structured-sparsity conversion and the
// layout-exploration model of SparStencil (arXiv 2506.22969, Section 3).
// Pure C++17, no HIP; the runtime turns a Layout into device tables.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ss {

constexpr int kZeta = -1;  // zero column (the paper's zero node)

// Morph geometry for one tile shape (Section 3.1; dimensions in Section 3.3).
struct Geometry {
    int ndim = 2;
    int k = 3;       // bounding-box width of the (possibly composed) stencil
    int r1 = 8;      // outputs crushed along x
    int r2 = 8;      // output rows crushed along y (1 in 1-D)
    int m_b = 0;     // row segments per patch plane: k + r2 - 1 (1 in 1-D)
    int g = 0;       // columns per row segment: k + r1 - 1
    int planes = 1;  // z planes per patch: k in 3-D
    int m_prime() const { return r1 * r2; }
    int k_prime() const { return planes * m_b * g; }
};

Geometry make_geometry(int ndim, int k, int r1, int r2);

// Structural nonzero test of A'[row, col]: the whole bounding box.
bool structural(const Geometry &gm, int row, int col);

// Staircase coefficient matrix A' (m' x k', row-major) for coefficients w
// of the bounding box (k^ndim, row-major).
std::vector<double> morph_matrix(const Geometry &gm, const std::vector<double> &w);

// Algorithm 1 on one plane: pairs of plane-local column indices
// (second = kZeta for a zero node), in construction order; zero count.
struct PairList {
    std::vector<std::pair<int, int>> pairs;
    int zeros = 0;
};
PairList two_level_matching(int m_blocks, int g, int k);

// Whole-matrix pair list: planes concatenated (3-D), offsets applied.
PairList matrix_pairs(const Geometry &gm);

// Group pairs into 4-wide groups [P0.a, P1.a, P0.b, P1.b] and pad with zero
// columns to a multiple of kfrag.
std::vector<int> group_pairs(const PairList &pl, int kfrag);

// Compressed values and positions (i0 < i1) per row and 4-group.  The
// positions kept are a row's structural ones (bounding box), or with
// by_value its nonzero ones (the kernels' compacted orders rely on that).
struct Compressed {
    std::vector<double> values;   // m' x K_pad/2
    std::vector<uint8_t> meta;    // m' x K_pad/4 x 2
};
bool compress(const Geometry &gm, const std::vector<double> &amat, const std::vector<int> &perm,
              Compressed *out, bool by_value = false);

// Round-to-nearest-even of an FP64 value into binary16 / bfloat16 bits.
// Returns false on overflow.
bool to_f16_bits(double x, uint16_t *bits);
bool to_bf16_bits(double x, uint16_t *bits);
double f16_value(uint16_t bits);
double bf16_value(uint16_t bits);

// Temporal fusion: S-fold self-composition of a correlation stencil.
std::vector<double> compose(const std::vector<double> &w, int ndim, int k, int steps, int *k_out);

// Layout-exploration model (Section 3.3, Eqs. 6-11).
struct ModelRow {
    int r1, r2;
    double t, t_compute, t_global, t_shared;
    int k_pad;
};
struct ModelParams {
    int ndim, k;
    int64_t dims[3];
    int elem_bytes, coef_bytes, passes, planes_state;
    int kfrag;
};
ModelRow model_time(const ModelParams &mp, int r1, int r2);
bool model_better(const ModelRow &a, const ModelRow &b);

// Structure-aware K order for the kernels (beyond the paper's bounding-box
// structure): a patch column is used
// when some row of A' holds a nonzero in it.  Sparse: the 4-groups of `perm`
// are kept when both their dominoes (slots 0-1 and 2-3, each a horizontally
// adjacent column pair) hold a used column, dropped when neither does, and
// the used dominoes of the remaining groups are re-paired first fit, in
// order, with the first later domino whose two columns share no nonzero row
// with theirs (else with a zero domino); kept groups first, then the new
// ones, zero groups up to a multiple of kfrag.  With an even patch row
// length g every kept half is also a domino (pc, pc+1) with pc even: a group
// with another half (Algorithm 1's in-block pairs (u, u+s2) with s2 odd) is
// taken apart into such dominoes, each once in order of first appearance,
// which join the re-pairing.  Dense: the column pairs
// (c, c+1), c even, of the natural order that hold a used column, zero
// columns up to a multiple of kfrag.  With every column used (box stencils)
// both return the plain orders.
std::vector<int> compact_groups(const Geometry &gm, const std::vector<double> &amat, const std::vector<int> &perm,
                                int kfrag);
std::vector<int> dense_order(const Geometry &gm, const std::vector<double> &amat, int kfrag);

// Every 32-bit B register of the sparse kernel holds two K slots that are
// either both zero columns or horizontally adjacent patch elements starting
// at an even column; only such layouts have a gather of 8-byte LDS reads.
bool pair_aligned(const Geometry &gm, const std::vector<int> &perm);

}  // namespace ss
