// FP32 SP2 product on FP32 MFMA: X_n^2 with FP32 operands and FP32
// accumulation over the whole K, and the SP2 update in FP32 (the FP32
// precision mode, and the FP32 tail of the BF16 hi + lo mode).
//
// The master X holds FP32 values in FP64 storage (X_0 is rounded by the
// first encode).  Before each product k_encode_f32 writes X_n as an FP32
// copy, so that the product streams 4-byte operands: at the FP32 matrix rate
// the 8-byte master would need twice the L2 bandwidth the FP64 product uses.
// One workgroup per upper 128 x 128 output tile, four waves of 64 x 64, each
// a 2 x 2 grid of v_mfma_f32_32x32x2f32 blocks; K is staged 32 rows at a time
// through LDS, double buffered.  The update X_{n+1} = P or 2 X_n - P is
// formed in FP32 and stored in the FP64 master, mirrored below the diagonal;
// the traces, the squared norm and the idempotency error are FP64 sums of
// the FP32 values.
#include <algorithm>
#include <type_traits>

#include "f32_internal.h"

namespace sp2 {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int FB = 128;   // output tile
constexpr int FK = 32;    // K rows per stage

// FP32 copy of X_n (phase 2 only): four elements per thread.
__global__ __launch_bounds__(256) void k_encode_f32(const double* __restrict__ buf0,
                                                    const double* __restrict__ buf1, size_t n4,
                                                    const State* __restrict__ st, float* __restrict__ x32) {
    if (st->done || st->phase != 2) return;
    const double* __restrict__ X = st->cur ? buf1 : buf0;
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n4; q += (size_t)gridDim.x * 256) {
        const double2 a = reinterpret_cast<const double2*>(X)[2 * q];
        const double2 b = reinterpret_cast<const double2*>(X)[2 * q + 1];
        reinterpret_cast<float4*>(x32)[q] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
    }
}

__global__ __launch_bounds__(256, 2) void k_gemm_f32(double* __restrict__ buf0, double* __restrict__ buf1,
                                                     int ld, const State* __restrict__ st,
                                                     const float* __restrict__ x32, double* __restrict__ part,
                                                     int tile_group) {
    if (st->done || st->phase != 2) return;
    // row k of a stage holds column c at (c + 32 (k & 1)) % 128: the two
    // half-waves of a fragment read (rows k and k + 1, 32 consecutive
    // columns each) then fall in disjoint LDS banks
    __shared__ float As[2][FK][FB];
    __shared__ float Bs[2][FK][FB];
    const int nt = ld / FB;
    int bi, bj;
    tile_of_block(blockIdx.x, nt, tile_group, bi, bj);
    const int t = tri_index(bi, bj, nt);
    const int i0 = bi * FB, j0 = bj * FB;
    double* __restrict__ Xn = st->cur ? buf0 : buf1;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wi = w >> 1, wj = w & 1;

    // X is symmetric, so P_ij = sum_k X_ki X_kj: both operands are row
    // segments of the FP32 copy (rows k, columns i0 .. i0 + 127 and
    // j0 .. j0 + 127).  Thread tid stages rows lrow + 8 s, columns lcol ..
    // lcol + 3.
    const int lrow = tid >> 5, lcol = 4 * (tid & 31);
    v4f ra[4], rb[4];
    auto gload = [&](int k0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const size_t off = (size_t)(k0 + lrow + 8 * s) * ld;
            ra[s] = *reinterpret_cast<const v4f*>(x32 + off + i0 + lcol);
            rb[s] = *reinterpret_cast<const v4f*>(x32 + off + j0 + lcol);
        }
    };
    auto sstore = [&](int stg) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int r = lrow + 8 * s;
            const int c = (lcol + 32 * (r & 1)) & (FB - 1);
            *reinterpret_cast<v4f*>(&As[stg][r][c]) = ra[s];
            *reinterpret_cast<v4f*>(&Bs[stg][r][c]) = rb[s];
        }
    };

    v16f acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[m][n][r] = 0.f;

    const int nk = ld / FK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int stg = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * FK);
#pragma unroll
        for (int k2 = 0; k2 < FK; k2 += 2) {
            // v_mfma_f32_32x32x2f32 operands: lane l holds A(row l % 32, k l / 32)
            // and B(k l / 32, column l % 32)
            const int kr = k2 + (lane >> 5);
            float a[2], b[2];
#pragma unroll
            for (int m = 0; m < 2; ++m) a[m] = As[stg][kr][(wi * 64 + m * 32 + (lane & 31) + 32 * (kr & 1)) & (FB - 1)];
#pragma unroll
            for (int n = 0; n < 2; ++n) b[n] = Bs[stg][kr][(wj * 64 + n * 32 + (lane & 31) + 32 * (kr & 1)) & (FB - 1)];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < 2; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m], b[n], acc[m][n], 0, 0, 0);
        }
        if (kt + 1 < nk) sstore(stg ^ 1);
        __syncthreads();
    }

    const int br = st->branch;
    const bool mirror = bi != bj;
    double tr = 0.0, fro = 0.0, idm = 0.0;
    // one straight-line body per mirrored flag (uniform): a per-element
    // branch on it keeps the addresses of every element live at once
    auto epilogue = [&](auto mirc) {
        constexpr bool MIR = decltype(mirc)::value;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                const int gj = j0 + wj * 64 + n * 32 + (lane & 31);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    // result: lane l, element r is row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
                    const int gi = i0 + wi * 64 + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const float p = acc[m][n][r];
                    const float x = x32[(size_t)gi * ld + gj];
                    const float xn = br ? 2.0f * x - p : p;
                    Xn[(size_t)gi * ld + gj] = (double)xn;
                    if constexpr (MIR) Xn[(size_t)gj * ld + gi] = (double)xn;
                    tr += gi == gj ? (double)xn : 0.0;
                    fro += (double)xn * (double)xn;
                    idm += ((double)p - (double)x) * ((double)p - (double)x);
                }
                // one 32 x 32 block at a time
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    if (mirror) epilogue(std::true_type{});
    else epilogue(std::false_type{});
    for (int o = 32; o > 0; o >>= 1) {
        tr += __shfl_xor(tr, o, 64);
        fro += __shfl_xor(fro, o, 64);
        idm += __shfl_xor(idm, o, 64);
    }
    __shared__ double red[3][4];
    if (lane == 0) {
        red[0][w] = tr;
        red[1][w] = fro;
        red[2][w] = idm;
    }
    __syncthreads();
    if (tid == 0) {
        const double wgt = mirror ? 2.0 : 1.0;
        part[3 * t + 0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        part[3 * t + 1] = wgt * ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
        part[3 * t + 2] = wgt * ((red[2][0] + red[2][1]) + (red[2][2] + red[2][3]));
    }
}

hipError_t launch_encode_f32(const double* buf0, const double* buf1, int ld, State* st, float* x32,
                             hipStream_t s) {
    const size_t n4 = (size_t)ld * ld / 4;
    const int grid = (int)std::min<size_t>((n4 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_encode_f32, dim3(grid), dim3(256), 0, s, buf0, buf1, n4, st, x32);
    return hipGetLastError();
}

hipError_t launch_gemm_f32(double* buf0, double* buf1, int ld, State* st, const float* x32, double* part,
                           int* nslots, int tile_group, hipStream_t s) {
    const int nt = ld / FB;
    const int T = tri_tiles(nt);
    *nslots = T;
    hipLaunchKernelGGL(k_gemm_f32, dim3(T), dim3(256), 0, s, buf0, buf1, ld, st, x32, part, tile_group);
    return hipGetLastError();
}

}  // namespace sp2
