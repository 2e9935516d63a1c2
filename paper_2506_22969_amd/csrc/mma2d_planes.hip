// 2-D MMA sweep kernels on a state of bfloat16 hi and lo planes (the planes
// are the B operands' hi and lo parts; bfloat16 coefficient parts).
#include "mma2d_impl.hpp"

namespace ss {

// Radius 1 (k = 3) at (8,8); radius 3 (k = 7): sparse (8,8) K 256, dense
// (8,4) K 160; radius 6 (k = 13, e.g. two fused radius-3 sweeps): (16,1),
// sparse and dense K 384, and sparse (16,2), K 448.  Star stencils use fewer
// patch columns: radius 3 sparse (8,8) K 192, dense (8,4) K 128; radius 6
// (two fused 13-point stars) sparse (16,1) and (16,2) K 320, dense (16,1)
// K 288.
static const MmaEntry kTable[] = {
    SS_MMA(8, 8, 2, 1, kSparse, kPartBF16, kStatePlanes),  SS_MMA(8, 8, 4, 1, kDense, kPartBF16, kStatePlanes),
    SS_MMA(8, 8, 4, 3, kSparse, kPartBF16, kStatePlanes),  SS_MMA(8, 4, 5, 3, kDense, kPartBF16, kStatePlanes),
    SS_MMA(16, 1, 6, 6, kSparse, kPartBF16, kStatePlanes), SS_MMA(16, 1, 12, 6, kDense, kPartBF16, kStatePlanes),
    SS_MMA(16, 2, 7, 6, kSparse, kPartBF16, kStatePlanes),
    SS_MMA(8, 8, 3, 3, kSparse, kPartBF16, kStatePlanes),  SS_MMA(8, 4, 4, 3, kDense, kPartBF16, kStatePlanes),
    SS_MMA(16, 1, 5, 6, kSparse, kPartBF16, kStatePlanes), SS_MMA(16, 1, 9, 6, kDense, kPartBF16, kStatePlanes),
    SS_MMA(16, 2, 5, 6, kSparse, kPartBF16, kStatePlanes),
};

const MmaEntry *mma_table_planes(int *n) {
    *n = (int)(sizeof kTable / sizeof kTable[0]);
    return kTable;
}

}  // namespace ss
