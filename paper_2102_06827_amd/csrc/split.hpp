// split.hpp -- compensated low-precision products for FP64-grade results:
// operand slicing (HBM-bound preparation) and the slice-pair matrix product.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "plan.hpp"

namespace comet {

struct SplitPlan {
  int mode = 0;             // 0: aligned BF16 slices, 1: BF16x3, 2: FP16x2, 3: aligned INT8 slices
  int S = 5;                // slices per operand
  int64_t Mp = 0, Np = 0, Kp = 0;   // padded matrix sizes of the packed operands
  size_t offA = 0, offB = 0, offEA = 0, offEB = 0;   // workspace byte offsets
  size_t offPA = 0, offPB = 0;                        // partial row exponents, ky per row
  int ky = 1;                                         // summation ranges of the exponent pass
  size_t ws_bytes = 0;
  int tile = 0;             // slice-pair product: 0 the 128 x 64 tile, 1 the 192 x 192 tile (modes 1, 2),
                            // 2 the 128 x 96 tile (mode 0, S <= 5)
};

// force_tile >= 0 sets the slice-pair tile (the autotuner's choice: 0 or 1
// for modes 1 and 2, 0 or 2 for mode 0); otherwise a size rule, which
// COMET_SPLIT_TILE overrides.
Status split_prepare(const Analysis &an, SplitPlan &sp, int force_tile = -1);
// vecA / vecB: the offset tables allow vector loads of the operand along its
// unit-stride dimension (the gather path's condition); the slicers use them
// where the operand's pointer is also 16-byte aligned.
hipError_t split_execute(const Analysis &an, const SplitPlan &sp, const GettTables &t, double alpha, const void *A,
                         const void *B, double beta, void *C, void *ws, hipStream_t s, bool vecA = false,
                         bool vecB = false);

}  // namespace comet
