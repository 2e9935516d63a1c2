// 2-D MMA sweep kernels on an FP32 state (split into binary16 or bfloat16
// hi + lo parts as it is gathered).
#include "mma2d_impl.hpp"

namespace ss {

// Radius 1 (k = 3) at tiles (8,8) and (16,4): sparse K 128 (2 chunks of 64),
// dense K 128 (4 chunks of 32).  Radius 3 (k = 7): sparse at (8,8), K 256;
// dense at (8,4), K 160; a 13-point star uses fewer patch columns: sparse
// K 192, dense K 128.  Radius 2 (k = 5, e.g. two fused radius-1 sweeps):
// sparse at (8,8), K 192; dense at (8,4), K 96.
static const MmaEntry kTable[] = {
    SS_MMA(8, 8, 2, 1, kSparse, kPartF16, kStateF32),  SS_MMA(8, 8, 4, 1, kDense, kPartF16, kStateF32),
    SS_MMA(16, 4, 2, 1, kSparse, kPartF16, kStateF32), SS_MMA(16, 4, 4, 1, kDense, kPartF16, kStateF32),
    SS_MMA(8, 8, 2, 1, kSparse, kPartBF16, kStateF32), SS_MMA(8, 8, 4, 1, kDense, kPartBF16, kStateF32),
    SS_MMA(16, 4, 2, 1, kSparse, kPartBF16, kStateF32), SS_MMA(16, 4, 4, 1, kDense, kPartBF16, kStateF32),
    SS_MMA(8, 8, 4, 3, kSparse, kPartF16, kStateF32),  SS_MMA(8, 4, 5, 3, kDense, kPartF16, kStateF32),
    SS_MMA(8, 8, 4, 3, kSparse, kPartBF16, kStateF32), SS_MMA(8, 4, 5, 3, kDense, kPartBF16, kStateF32),
    SS_MMA(8, 8, 3, 3, kSparse, kPartF16, kStateF32),  SS_MMA(8, 4, 4, 3, kDense, kPartF16, kStateF32),
    SS_MMA(8, 8, 3, 3, kSparse, kPartBF16, kStateF32), SS_MMA(8, 4, 4, 3, kDense, kPartBF16, kStateF32),
    SS_MMA(8, 8, 3, 2, kSparse, kPartF16, kStateF32),  SS_MMA(8, 4, 3, 2, kDense, kPartF16, kStateF32),
    SS_MMA(8, 8, 3, 2, kSparse, kPartBF16, kStateF32), SS_MMA(8, 4, 3, 2, kDense, kPartBF16, kStateF32),
};

const MmaEntry *mma_table_f32(int *n) {
    *n = (int)(sizeof kTable / sizeof kTable[0]);
    return kTable;
}

}  // namespace ss
