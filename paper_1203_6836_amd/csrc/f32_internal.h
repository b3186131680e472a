// Internal declaration of the FP32 SP2 product (gemm_f32.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "sp2_internal.h"

namespace sp2 {

// One SP2 product X_n^2 on FP32 MFMA with the fused update, for states in
// phase 2 (the FP32 precision, and the FP32 tail of the BF16 hi + lo mode);
// other states return at once.  One workgroup per upper 128 x 128 tile (T =
// nt (nt + 1) / 2, written to *nslots, one partial slot each); tile_group is
// the super-tile size of the tile order.  ld is a multiple of 128.
hipError_t launch_gemm_f32(double* buf0, double* buf1, int ld, State* st, double* part, int* nslots,
                           int tile_group, hipStream_t s);

}  // namespace sp2
