// 2-D MMA sweep kernels on a plain binary16 state: binary16 coefficients and
// state in one product per K chunk, FP32 accumulation, binary16 results.
#include "mma2d_conv.hpp"

namespace ss {

// The tiles and K chunk counts of the FP32-state tables for radius 1 to 3
// ((8,8), (8,4), and (16,4) at radius 1), sparse and dense.
static const MmaEntry kTable[] = {
    SS_MMA_CONV(8, 8, 2, 1, kSparse, kPartF16, kStateF16),
    SS_MMA_CONV(8, 4, 1, 1, kSparse, kPartF16, kStateF16),
    SS_MMA_CONV(16, 4, 2, 1, kSparse, kPartF16, kStateF16),
    SS_MMA_CONV(8, 8, 4, 1, kDense, kPartF16, kStateF16),
    SS_MMA_CONV(8, 4, 2, 1, kDense, kPartF16, kStateF16),
    SS_MMA_CONV(8, 8, 3, 2, kSparse, kPartF16, kStateF16),
    SS_MMA_CONV(8, 8, 2, 2, kSparse, kPartF16, kStateF16),
    SS_MMA_CONV(8, 4, 2, 2, kSparse, kPartF16, kStateF16),
    SS_MMA_CONV(8, 4, 3, 2, kDense, kPartF16, kStateF16),
    SS_MMA_CONV(8, 8, 4, 3, kSparse, kPartF16, kStateF16),
    SS_MMA_CONV(8, 8, 3, 3, kSparse, kPartF16, kStateF16),
    SS_MMA_CONV(8, 4, 3, 3, kSparse, kPartF16, kStateF16),
    SS_MMA_CONV(8, 4, 2, 3, kSparse, kPartF16, kStateF16),
    SS_MMA_CONV(8, 4, 5, 3, kDense, kPartF16, kStateF16),
    SS_MMA_CONV(8, 4, 4, 3, kDense, kPartF16, kStateF16),
};

const MmaEntry *mma_table_f16(int *n) {
    *n = (int)(sizeof kTable / sizeof kTable[0]);
    return kTable;
}

}  // namespace ss
