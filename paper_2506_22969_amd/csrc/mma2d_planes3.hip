// 2-D MMA sweep kernels on a state of bfloat16 hi, mid and lo planes (the
// planes are the B operands' three parts; three-part bfloat16 coefficients;
// six products per K chunk).
#include "mma2d_conv.hpp"

namespace ss {

// One M-block tiles (16 outputs: (8,2) and (16,1)), whose three sets of A
// fragments fit the register file.  Radius 1 (k = 3): sparse K 64 at (8,2);
// dense K 64 at (8,2).  Radius 3 (k = 7): sparse K 128 at (8,2); dense K 128
// at (8,2) (13-point star: 96).  Radius 6 (k = 13, e.g. two fused radius-3
// sweeps): sparse K 384 at (8,2) and (16,1) (two fused 13-point stars: 192
// and 320); dense K 288 at (8,2) (stars: 192) and 384 at (16,1) (288).
static const MmaEntry kTable[] = {
    SS_MMA_CONV(8, 2, 1, 1, kSparse, kPartBF16, kStatePlanes3),  SS_MMA_CONV(8, 2, 2, 1, kDense, kPartBF16, kStatePlanes3),
    SS_MMA_CONV(8, 2, 2, 3, kSparse, kPartBF16, kStatePlanes3),  SS_MMA_CONV(8, 2, 4, 3, kDense, kPartBF16, kStatePlanes3),
    SS_MMA_CONV(8, 2, 3, 3, kDense, kPartBF16, kStatePlanes3),
    SS_MMA_CONV(8, 2, 6, 6, kSparse, kPartBF16, kStatePlanes3),  SS_MMA_CONV(8, 2, 3, 6, kSparse, kPartBF16, kStatePlanes3),
    SS_MMA_CONV(16, 1, 6, 6, kSparse, kPartBF16, kStatePlanes3), SS_MMA_CONV(16, 1, 5, 6, kSparse, kPartBF16, kStatePlanes3),
    SS_MMA_CONV(8, 2, 9, 6, kDense, kPartBF16, kStatePlanes3),   SS_MMA_CONV(8, 2, 6, 6, kDense, kPartBF16, kStatePlanes3),
    SS_MMA_CONV(16, 1, 12, 6, kDense, kPartBF16, kStatePlanes3), SS_MMA_CONV(16, 1, 9, 6, kDense, kPartBF16, kStatePlanes3),
};

const MmaEntry *mma_table_planes3(int *n) {
    *n = (int)(sizeof kTable / sizeof kTable[0]);
    return kTable;
}

}  // namespace ss
