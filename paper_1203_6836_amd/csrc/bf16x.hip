// BF16 hi + lo split SP2 product with FP32 accumulation (the configured
// mixed-precision recipe, kept as a measured mode).
//
// The master X holds FP32 values.  Each product encodes x = X_ij as
// hi = bf16(x), lo = bf16(x - hi) (round to nearest even) and forms
// X^2 ~ hi hi^T + hi lo^T + lo hi^T on v_mfma_f32_32x32x16_bf16 with one FP32
// accumulator over the whole K; the update X_{n+1} = P or 2X - P is done in
// FP32 and stored back as FP32 values.  Traces, norms, branch and stop stay
// FP64.
//
// Storage mirrors the int8 digit planes: 1 KiB blocks of 32 rows x 16 k
// (bf16), row-major over blocks (ld / 16 per block row); inside a block row r
// holds two 16-byte halves (k % 16 < 8 and >= 8) swapped when swz(r) = 1, so
// the MFMA fragment reads (lane l: row l % 32, k-half l / 32) are free of bank
// conflicts.  Tile 128 x 128, 8 waves of 32 x 64, K staged 32 at a time.
#include "split_internal.h"

namespace sp2 {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int bswz(int r) { return ((r >> 2) ^ (r >> 3)) & 1; }

// Round-to-nearest-even float -> bf16 bit pattern (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

// One wave per padded row: hi and lo planes of the FP32 value of X_n.
__global__ __launch_bounds__(256) void k_encode_bf16(const double* __restrict__ buf0,
                                                     const double* __restrict__ buf1, int ld,
                                                     const State* __restrict__ st,
                                                     uint16_t* __restrict__ planes) {
    if (st->done || st->phase != 1) return;
    const double* X = st->cur ? buf1 : buf0;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const double* row = X + (size_t)i * ld;
    const size_t plane = (size_t)ld * ld;
    const size_t rowblk = (size_t)(i >> 5) * (ld >> 4);
    const int r32 = i & 31;
    for (int j = 8 * lane; j < ld; j += 512) {
        uint32_t h[8], l[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float x = (float)row[j + q];
            h[q] = bf16_bits(x);
            l[q] = bf16_bits(x - bf16_value(h[q]));
        }
        const size_t off = (rowblk + (j >> 4)) * 512 + r32 * 16 + 8 * (((j >> 3) & 1) ^ bswz(r32));
        uint4 vh, vl;
        vh.x = h[0] | (h[1] << 16); vh.y = h[2] | (h[3] << 16); vh.z = h[4] | (h[5] << 16); vh.w = h[6] | (h[7] << 16);
        vl.x = l[0] | (l[1] << 16); vl.y = l[2] | (l[3] << 16); vl.z = l[4] | (l[5] << 16); vl.w = l[6] | (l[7] << 16);
        *reinterpret_cast<uint4*>(planes + off) = vh;
        *reinterpret_cast<uint4*>(planes + plane + off) = vl;
    }
}

constexpr int BB = 128;           // tile

struct BfSmem {
    // [stage][op * 2 * 2 * 4 + plane * 8 + kblock * 4 + row block][1 KiB]
    uint16_t buf[2][32][512];
};

__global__ __launch_bounds__(512) void k_gemm_bf16x2(double* __restrict__ buf0, double* __restrict__ buf1,
                                                     int ld, const State* __restrict__ st,
                                                     const uint16_t* __restrict__ planes,
                                                     double* __restrict__ part, int tile_group) {
    if (st->done || st->phase != 1) return;
    extern __shared__ __align__(16) uint16_t bsm_raw[];
    BfSmem& sm = *reinterpret_cast<BfSmem*>(bsm_raw);
    const int nt = ld / BB;
    int bi, bj;
    tile_of_block(blockIdx.x, nt, tile_group, bi, bj);
    const int t = tri_index(bi, bj, nt);
    const int i0 = bi * BB, j0 = bj * BB;
    const double* __restrict__ Xc = st->cur ? buf1 : buf0;
    double* __restrict__ Xn = st->cur ? buf0 : buf1;
    const size_t plane = (size_t)ld * ld;
    const int nb = ld >> 4;                  // 16-wide k blocks per block row
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;

    // stage = 32 k: 2 operands x 2 planes x 2 k blocks x 4 row blocks = 32 KiB-blocks
    v4i pre[4];
    auto gload = [&](int kt) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int c = tid + 512 * m;      // 0 .. 2047 sixteen-byte chunks
            const int blk = c >> 6;           // 0 .. 31
            const int op = blk >> 4, pl = (blk >> 3) & 1, kb = (blk >> 2) & 1, rb = blk & 3;
            const int grb = ((op ? j0 : i0) >> 5) + rb;
            pre[m] = *reinterpret_cast<const v4i*>(planes + pl * plane +
                                                   ((size_t)grb * nb + 2 * kt + kb) * 512 + 8 * (c & 63));
        }
    };
    auto sstore = [&](int stg) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int c = tid + 512 * m;
            *reinterpret_cast<v4i*>(&sm.buf[stg][c >> 6][8 * (c & 63)]) = pre[m];
        }
    };
    v16f acc[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.f;
    const int fr = lane & 31;
    const int foff = fr * 16 + 8 * ((lane >> 5) ^ bswz(fr));   // in bf16 elements
    const int nk = ld / 32;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int stg = kt & 1;
        if (kt + 1 < nk) gload(kt + 1);
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            v8bf a[2], b[2][2];
#pragma unroll
            for (int pl = 0; pl < 2; ++pl) {
                a[pl] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4i*>(&sm.buf[stg][pl * 8 + kb * 4 + wr][foff]));
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    b[pl][c] = __builtin_bit_cast(
                        v8bf, *reinterpret_cast<const v4i*>(&sm.buf[stg][16 + pl * 8 + kb * 4 + wc * 2 + c][foff]));
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[0][c], acc[c], 0, 0, 0);   // lo hi
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[1][c], acc[c], 0, 0, 0);   // hi lo
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[0][c], acc[c], 0, 0, 0);   // hi hi
            }
        }
        if (kt + 1 < nk) sstore(stg ^ 1);
        __syncthreads();
    }

    const int br = st->branch;
    const bool mirror = bi != bj;
    double tr = 0.0, fro = 0.0, idm = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int gj = j0 + wc * 64 + c * 32 + (lane & 31);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            // v_mfma_f32_32x32x16_bf16 result: lane l, element r is row 8 (r/4) + 4 (l/32) + r%4, column l%32
            const int gi = i0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const float p = acc[c][r];
            const float x = (float)Xc[(size_t)gi * ld + gj];
            const float xn = br ? 2.0f * x - p : p;
            Xn[(size_t)gi * ld + gj] = (double)xn;
            if (mirror) Xn[(size_t)gj * ld + gi] = (double)xn;
            if (gi == gj) tr += (double)xn;
            fro += (double)xn * (double)xn;
            idm += ((double)p - (double)x) * ((double)p - (double)x);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        tr += __shfl_xor(tr, o, 64);
        fro += __shfl_xor(fro, o, 64);
        idm += __shfl_xor(idm, o, 64);
    }
    __shared__ double red[3][8];
    if (lane == 0) {
        red[0][w] = tr;
        red[1][w] = fro;
        red[2][w] = idm;
    }
    __syncthreads();
    if (tid == 0) {
        double s3[3];
        for (int q = 0; q < 3; ++q)
            s3[q] = ((red[q][0] + red[q][1]) + (red[q][2] + red[q][3])) +
                    ((red[q][4] + red[q][5]) + (red[q][6] + red[q][7]));
        const double wgt = mirror ? 2.0 : 1.0;
        part[3 * t + 0] = s3[0];
        part[3 * t + 1] = wgt * s3[1];
        part[3 * t + 2] = wgt * s3[2];
    }
}

hipError_t launch_bf16x2_encode(SplitScratch& s, const double* buf0, const double* buf1, int ld, State* st,
                                hipStream_t stream) {
    hipLaunchKernelGGL(k_encode_bf16, dim3(ld / 4), dim3(256), 0, stream, buf0, buf1, ld, st, s.bf);
    return hipGetLastError();
}

hipError_t launch_bf16x2_gemm(SplitScratch& s, double* buf0, double* buf1, int ld, State* st, double* part,
                              int* nslots, hipStream_t stream) {
    const int nt = ld / BB;
    const int T = nt * (nt + 1) / 2;
    *nslots = T;
    static std::atomic<unsigned long long> attr_done{0};
    hipError_t e = once_per_device(attr_done, [] {
        return hipFuncSetAttribute((const void*)k_gemm_bf16x2, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)sizeof(BfSmem));
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gemm_bf16x2, dim3(T), dim3(512), sizeof(BfSmem), stream, buf0, buf1, ld, st, s.bf, part,
                       s.tile_group);
    return hipGetLastError();
}

}  // namespace sp2
