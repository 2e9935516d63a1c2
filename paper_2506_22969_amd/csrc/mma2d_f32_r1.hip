// 2-D MMA sweep kernels on an FP32 state (split into binary16 or bfloat16
// hi + lo parts once per work item), radius 1.
#include "mma2d_conv.hpp"

namespace ss {

// Radius 1 (k = 3): sparse K 128 at (8,8), (16,4) and (16,2), K 64 at (8,4)
// and (8,2); dense K 128 at (8,8) and (16,4), K 64 at (8,4).
static const MmaEntry kTable[] = {
    SS_MMA_CONV(8, 8, 2, 1, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(16, 4, 2, 1, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 4, 1, 1, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(16, 2, 2, 1, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 2, 1, 1, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 8, 4, 1, kDense, kPartF16, kStateF32),
    SS_MMA_CONV(16, 4, 4, 1, kDense, kPartF16, kStateF32),
    SS_MMA_CONV(8, 4, 2, 1, kDense, kPartF16, kStateF32),
    SS_MMA_CONV(8, 8, 2, 1, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(16, 4, 2, 1, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 4, 1, 1, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(16, 2, 2, 1, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 2, 1, 1, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 8, 4, 1, kDense, kPartBF16, kStateF32),
    SS_MMA_CONV(16, 4, 4, 1, kDense, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 4, 2, 1, kDense, kPartBF16, kStateF32),
};

const MmaEntry *mma_table_f32_r1(int *n) {
    *n = (int)(sizeof kTable / sizeof kTable[0]);
    return kTable;
}

}  // namespace ss
