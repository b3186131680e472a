// Internal declarations of the general FP64 product kernel (gemm_f64.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace sp2 {

// C = alpha A^T B + beta C_in + gamma I over N x N row-major matrices with
// leading dimension N.  C_in may be null when beta == 0, and may be C.  A, B
// must not alias C.
struct GemmTN {
    const double* A;
    const double* B;
    const double* Cin;
    double* C;
    int N;
    double alpha, beta, gamma;
};

// sym: A^T B is symmetric (the caller's assertion): only the upper tiles are
// formed and mirrored.  chunk (chunk_bytes, may be null: no K split): the
// chunk accumulators of split tiles (kF64Chunk doubles each).  tile_group:
// super-tile size of the tile order (8 is a good default).
hipError_t launch_gemm_tn(const GemmTN& g, bool sym, int tile_group, double* chunk, size_t chunk_bytes,
                          hipStream_t s);

}  // namespace sp2
