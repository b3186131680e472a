// Roofline denominator measured on the device: an int8 matrix-core loop with
// no memory traffic.  Not a step of the SP2 path; sp2_int8_mfma_rate times it.
//
// Each wave keeps four independent accumulator chains busy with the
// instruction of the int8 product kernel.  Its rate depends on the data: zero
// operands run near the nominal peak, nonzero operands settle far lower (the
// clock is power-limited), so the operands are pseudo-random balanced 7-bit
// digits, the range of the digit planes, whose low six bits flip between
// consecutive products.
#include <hip/hip_runtime.h>

#include "sp2_internal.h"

namespace sp2 {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ unsigned xorshift(unsigned& h) {
    h ^= h << 13;
    h ^= h >> 17;
    h ^= h << 5;
    return h;
}

// int8: 4 chains of v_mfma_i32_32x32x32_i8 (65536 ops each) per iteration.
// Bytes of a, b in [-64, 63]; the masks touch bits 0-5 only, which keeps
// every byte on its side of zero and so in range.
__global__ __launch_bounds__(256) void k_peak_i8(int iters, double* __restrict__ out) {
    unsigned h = (blockIdx.x * 256u + threadIdx.x + 1u) * 0x9E3779B9u;
    v4i a, b, fa, fb;
    auto digits = [&]() {   // four bytes (r & 0x7f) - 64
        const unsigned r = xorshift(h);
        unsigned v = 0;
        for (int k = 0; k < 4; ++k) v |= (unsigned)(uint8_t)((int)((r >> (8 * k)) & 0x7fu) - 64) << (8 * k);
        return (int)v;
    };
    for (int q = 0; q < 4; ++q) {
        a[q] = digits();
        b[q] = digits();
        fa[q] = (int)(xorshift(h) & 0x3f3f3f3fu);
        fb[q] = (int)(xorshift(h) & 0x3f3f3f3fu);
    }
    v16i c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b, a, c1, 0, 0, 0);
        a ^= fa;
        b ^= fb;
        c2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b, a, c3, 0, 0, 0);
        a ^= fb;
        b ^= fa;
    }
    unsigned s = 0;
    for (int r = 0; r < 16; ++r) s += (unsigned)c0[r] + (unsigned)c1[r] + (unsigned)c2[r] + (unsigned)c3[r];
    if (s == 0x2468ACE1u) out[0] = (double)s;   // keeps the chains live; practically never taken
}

hipError_t launch_int8_rate(int grid, int iters, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_peak_i8, dim3(grid), dim3(256), 0, stream, iters, out);
    return hipGetLastError();
}

}  // namespace sp2
