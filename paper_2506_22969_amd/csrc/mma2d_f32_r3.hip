// 2-D MMA sweep kernels on an FP32 state (split into binary16 or bfloat16
// hi + lo parts once per work item), radius 3.
#include "mma2d_conv.hpp"

namespace ss {

// Radius 3 (k = 7, e.g. three fused radius-1 sweeps): sparse K 256 at (8,8)
// (K 192 for a 13-point star), K 192 at (8,4) (star: 128) and (16,2), K 128
// at (8,2); dense K 160 at (8,4) (star: 128).
static const MmaEntry kTable[] = {
    SS_MMA_CONV(8, 8, 4, 3, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 8, 3, 3, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 4, 3, 3, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 4, 2, 3, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(16, 2, 3, 3, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 2, 2, 3, kSparse, kPartF16, kStateF32),
    SS_MMA_CONV(8, 4, 5, 3, kDense, kPartF16, kStateF32),
    SS_MMA_CONV(8, 4, 4, 3, kDense, kPartF16, kStateF32),
    SS_MMA_CONV(8, 8, 4, 3, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 8, 3, 3, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 4, 3, 3, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 4, 2, 3, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(16, 2, 3, 3, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 2, 2, 3, kSparse, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 4, 5, 3, kDense, kPartBF16, kStateF32),
    SS_MMA_CONV(8, 4, 4, 3, kDense, kPartBF16, kStateF32),
};

const MmaEntry *mma_table_f32_r3(int *n) {
    *n = (int)(sizeof kTable / sizeof kTable[0]);
    return kTable;
}

}  // namespace ss
