// 2-D MMA sweep kernels on an FP32 state (split into binary16 or bfloat16
// hi + lo parts once per work item), radius 2.
#include "mma2d_conv.hpp"

namespace ss {

// Radius 2 (k = 5, e.g. two fused radius-1 sweeps): sparse K 192 at (8,8)
// (K 128 for a 9-point star), K 128 at (8,4), (16,2) and (8,2) (K 64 for a
// star at (8,2)); dense K 96 at (8,4).
static const MmaEntry kTable[] = {
    SS_MMA_CONV(8, 8, 3, 2, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 8, 2, 2, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 4, 2, 2, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(16, 2, 2, 2, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 2, 2, 2, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 2, 1, 2, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 4, 3, 2, kDense, kPartF16, kStateF32),
    SS_MMA_CONV(8, 8, 3, 2, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 8, 2, 2, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 4, 2, 2, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(16, 2, 2, 2, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 2, 2, 2, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 2, 1, 2, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 4, 3, 2, kDense, kPartBF16, kStateF32),
};

const MmaEntry *mma_table_f32_r2(int *n) {
    *n = (int)(sizeof kTable / sizeof kTable[0]);
    return kTable;
}

}  // namespace ss
