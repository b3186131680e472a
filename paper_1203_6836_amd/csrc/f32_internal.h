// Internal declaration of the FP32 SP2 product (gemm_f32.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "sp2_internal.h"

namespace sp2 {

// For states in phase 2 (the FP32 precision, and the FP32 tail of the BF16
// hi + lo mode; other states return at once):
// launch_encode_f32 writes X_n (the current FP64 master buffer, ld x ld) as
// FP32 into x32 (ld x ld floats);
// launch_gemm_f32 forms X_n^2 from x32 on FP32 MFMA with the fused update
// into the other master buffer, one workgroup per upper 128 x 128 tile (T =
// nt (nt + 1) / 2, written to *nslots, one partial slot each); tile_group is
// the super-tile size of the tile order.  ld is a multiple of 128.
hipError_t launch_encode_f32(const double* buf0, const double* buf1, int ld, State* st, float* x32,
                             hipStream_t s);
hipError_t launch_gemm_f32(double* buf0, double* buf1, int ld, State* st, const float* x32, double* part,
                           int* nslots, int tile_group, hipStream_t s);

}  // namespace sp2
