// 2-D MMA sweep kernels on a state of bfloat16 hi and lo planes (the planes
// are the B operands' hi and lo parts; bfloat16 coefficient parts).
#include "mma2d_conv.hpp"

namespace ss {

// Radius 1 (k = 3): sparse K 128 at (8,8), K 64 at (8,4) and (8,2); dense K
// 128 at (8,8), 64 at (8,4).  Radius 3 (k = 7): sparse K 256 at (8,8), 192
// at (8,4) and (16,2), 128 at (8,2) (13-point star: 192 at (8,8), 128 at
// (8,4)); dense K 160 at (8,4) (star: 128).  Radius 6 (k = 13, e.g. two
// fused radius-3 sweeps): sparse K 448 at (16,2) and (8,4), 384 at (16,1)
// and (8,2) (two fused 13-point stars: 320 at (16,2) and (16,1), 256 at
// (8,4), 192 at (8,2)); dense K 384 at (16,1), 288 at (8,2) (stars: 288 and
// 192).
static const MmaEntry kTable[] = {
    SS_MMA_CONV(8, 8, 2, 1, kSparse, kPartBF16, kStatePlanes),  SS_MMA_CONV(8, 4, 1, 1, kSparse, kPartBF16, kStatePlanes),
    SS_MMA_CONV(8, 2, 1, 1, kSparse, kPartBF16, kStatePlanes),  SS_MMA_CONV(8, 8, 4, 1, kDense, kPartBF16, kStatePlanes),
    SS_MMA_CONV(8, 4, 2, 1, kDense, kPartBF16, kStatePlanes),
    SS_MMA_CONV(8, 8, 4, 3, kSparse, kPartBF16, kStatePlanes),  SS_MMA_CONV(8, 8, 3, 3, kSparse, kPartBF16, kStatePlanes),
    SS_MMA_CONV(8, 4, 3, 3, kSparse, kPartBF16, kStatePlanes),  SS_MMA_CONV(8, 4, 2, 3, kSparse, kPartBF16, kStatePlanes),
    SS_MMA_CONV(8, 2, 2, 3, kSparse, kPartBF16, kStatePlanes),  SS_MMA_CONV(16, 2, 3, 3, kSparse, kPartBF16, kStatePlanes),
    SS_MMA_CONV(8, 4, 5, 3, kDense, kPartBF16, kStatePlanes),   SS_MMA_CONV(8, 4, 4, 3, kDense, kPartBF16, kStatePlanes),
    SS_MMA_CONV(16, 2, 7, 6, kSparse, kPartBF16, kStatePlanes), SS_MMA_CONV(16, 2, 5, 6, kSparse, kPartBF16, kStatePlanes),
    SS_MMA_CONV(16, 1, 6, 6, kSparse, kPartBF16, kStatePlanes), SS_MMA_CONV(16, 1, 5, 6, kSparse, kPartBF16, kStatePlanes),
    SS_MMA_CONV(8, 2, 6, 6, kSparse, kPartBF16, kStatePlanes),  SS_MMA_CONV(8, 2, 3, 6, kSparse, kPartBF16, kStatePlanes),
    SS_MMA_CONV(8, 4, 7, 6, kSparse, kPartBF16, kStatePlanes),  SS_MMA_CONV(8, 4, 4, 6, kSparse, kPartBF16, kStatePlanes),
    SS_MMA_CONV(16, 1, 12, 6, kDense, kPartBF16, kStatePlanes), SS_MMA_CONV(16, 1, 9, 6, kDense, kPartBF16, kStatePlanes),
    SS_MMA_CONV(8, 2, 9, 6, kDense, kPartBF16, kStatePlanes),   SS_MMA_CONV(8, 2, 6, 6, kDense, kPartBF16, kStatePlanes),
};

const MmaEntry *mma_table_planes(int *n) {
    *n = (int)(sizeof kTable / sizeof kTable[0]);
    return kTable;
}

}  // namespace ss
