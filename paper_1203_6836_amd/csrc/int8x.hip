// Reduced-precision SP2 product on int8 MFMA with exact integer accumulation
// (an error-free split of FP64 operands into integer slices whose products
// are exact in integer arithmetic, the Ozaki scheme for matrix products).
//
// The FP64 master X_n is split row by row into fixed-point digit planes:
// with the row scale s_i = (1 + 2^-7) max_j |X_ij| (row_scale), y = X_ij / s_i
// lies in [-0.993, 0.993] and is written as y ~ sum_t d_t 2^-(e0 + W t), W
// bits per digit (digit_bits), e0 = W - 1:
//   W = 8: the integer m = rint(y 2^(8S - 1)) (|m| < 0.9961 2^(8S - 1), the
//     range of the excess code below) is written in base 256 with digits in
//     [-128, 127]: the bytes of m + 0x80..80 (S bytes), each read back as a
//     byte minus 128.  One rounding, error <= 2^-(8S) s_i; the top digit
//     uses its whole byte, since the row maximum sits just inside the range
//     (a power-of-two scale would leave it between 1/4 and 1/2 of it, one
//     to two bits less per operand);
//   W = 7: digits |d_t| <= 64 taken by successive round-to-nearest of the
//     remainder (each remainder exact in FP64) with weights 2^-(6 + 7 t), 7
//     bits a digit, for larger K.
// Because X is symmetric,
//     (X^2)_ij = sum_k X_ik X_jk ~ s_i s_j sum_{t,u} 2^-(2 e0 + W(t+u)) sum_k d_t[i,k] d_u[j,k],
// i.e. every digit product reads contiguous rows of the digit planes for both
// operands.  Products of planes t, u < S with level L = t + u < NL are kept,
// NL = S (the triangle) or S + 1 (the next level's products of the inner
// planes too: with 8-bit digits this is the accuracy of rounding each
// operand to 8S bits, for S - 1 more products).  Those of one level share an
// int32 accumulator, which is exact: a level has at most S products, and
// W = 8: |acc| <= S 2^14 K < 2^31 by the choice of W; W = 7: |d| <= 64,
// K <= 65536.  Levels are combined in FP64 in the epilogue, which then
// applies the SP2 update exactly like the FP64 product.  The plane count may
// change from product to product (the host picks each launch's), so the
// digit width is a function of (ld, S) that encode and product agree on.
//
// Work layout, storage and staging: see the comments at the kernels.
#include <atomic>
#include <algorithm>

#include "split_internal.h"

namespace sp2 {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ double wred_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wred_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Digit planes are stored blocked: plane t, row i, column j lives in the
// 1 KiB block (i / 32, j / 32) (blocks row-major, ld / 32 per block row), at
// byte (i % 32) * 32 + 16 * (((j / 16) % 2) ^ swz(i % 32)) + j % 16.  One
// block is one MFMA operand fragment for 32 rows and 32 k: a wave stages it
// with one contiguous 16-byte-per-lane load, and the swizzle
// swz(r) = ((r >> 2) ^ (r >> 3)) & 1 makes the fragment reads (lane l: row
// l % 32, k-half l / 32) free of LDS bank conflicts.
__device__ __forceinline__ int dswz(int r) { return ((r >> 2) ^ (r >> 3)) & 1; }

// --------------------------------------------------------------- encoding
// Bits per digit of an S-plane split of operands with K = ld: 8 while every
// level accumulator provably fits int32 (at most S products of |d| <= 128
// per level), else 7.
__host__ __device__ __forceinline__ int digit_bits(int ld, int S) {
    return (long long)S * 16384LL * ld < 2147483648LL ? 8 : 7;
}
// Exponent of the top digit's weight, 2^-e0.
__host__ __device__ __forceinline__ int digit_e0(int W) { return W == 8 ? 7 : 6; }

// Row scale s = (1 + 2^-7) m of a row with maximum m (1 for a zero row) and
// its reciprocal, the factor that maps the row into [-0.993, 0.993] (one
// rounding each: |X_ij| inv <= (1 + 2^-51) / (1 + 2^-7)).  Every encoder
// takes both from here, so they agree bit for bit.
__device__ __forceinline__ double row_scale(double m, double* s_out) {
    const double s = m > 0.0 ? m * 1.0078125 : 1.0;
    if (s_out) *s_out = s;
    return 1.0 / s;
}

// W = 8: m + 0x80..80 (S bytes) for m = rint(y 2^(8S - 1)), |y| <= 0.993 (so
// -0x80..80 <= m < 0x7F..7F80, the range whose excess code has S bytes);
// byte S - 1 - t of it XOR 0x80 is digit t as an int8.
__device__ __forceinline__ unsigned long long excess_digits(double y, int S) {
    const long long m = (long long)rint(y * ldexp(1.0, 8 * S - 1));
    return (unsigned long long)m + (0x8080808080808080ull >> (8 * (8 - S)));
}
__device__ __forceinline__ unsigned excess_digit(unsigned long long u, int S, int t) {
    return (unsigned)((u >> (8 * (S - 1 - t))) & 0xFFull) ^ 0x80u;
}

// Digits of eight values y (|y| <= 0.993) into eight packed bytes per plane.
template <int S>
__device__ __forceinline__ void pack_digits8(double (&y)[8], int W, unsigned long long (&packed)[S]) {
    if (W == 8) {
        unsigned long long u[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) u[q] = excess_digits(y[q], S);
#pragma unroll
        for (int t = 0; t < S; ++t) {
            unsigned long long p = 0ull;
#pragma unroll
            for (int q = 0; q < 8; ++q) p |= (unsigned long long)excess_digit(u[q], S, t) << (8 * q);
            packed[t] = p;
        }
        return;
    }
#pragma unroll
    for (int t = 0; t < S; ++t) {
        const double w = ldexp(1.0, 6 + 7 * t);      // digit weight 2^-(6+7t)
        const double iw = ldexp(1.0, -(6 + 7 * t));
        unsigned long long p = 0ull;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double d = rint(y[q] * w);        // |d| <= 64
            y[q] -= d * iw;                          // exact remainder
            p |= (unsigned long long)(uint8_t)(int8_t)d << (8 * q);
        }
        packed[t] = p;
    }
}

// One wave per padded row: row scale and `slices` digit planes of columns
// [c0, c1) (multiples of 32; the row is zero outside them).
template <int S>
__device__ __forceinline__ void encode_row(const double* __restrict__ X, int ld, int i, int lane, int8_t* __restrict__ digits,
                           double* __restrict__ scale, int c0, int c1) {
    const double* row = X + (size_t)i * ld;
    const int W = digit_bits(ld, S);
    double m = 0.0;
    for (int j = c0 + 8 * lane; j < c1; j += 512) {
        const double4 a = *reinterpret_cast<const double4*>(row + j);
        const double4 b = *reinterpret_cast<const double4*>(row + j + 4);
        m = fmax(m, fmax(fmax(fabs(a.x), fabs(a.y)), fmax(fabs(a.z), fabs(a.w))));
        m = fmax(m, fmax(fmax(fabs(b.x), fabs(b.y)), fmax(fabs(b.z), fabs(b.w))));
    }
    m = wred_max(m);
    double sc;
    const double inv = row_scale(m, &sc);
    if (lane == 0) scale[i] = sc;
    const size_t plane = (size_t)ld * ld;
    const size_t rowblk = (size_t)(i >> 5) * (ld >> 5);
    const int r32 = i & 31;
    for (int j = c0 + 8 * lane; j < c1; j += 512) {
        double y[8];
        const double4 a = *reinterpret_cast<const double4*>(row + j);
        const double4 b = *reinterpret_cast<const double4*>(row + j + 4);
        y[0] = a.x * inv; y[1] = a.y * inv; y[2] = a.z * inv; y[3] = a.w * inv;
        y[4] = b.x * inv; y[5] = b.y * inv; y[6] = b.z * inv; y[7] = b.w * inv;
        const size_t off = (rowblk + (j >> 5)) * 1024 + r32 * 32 + 16 * (((j >> 4) & 1) ^ dswz(r32)) + (j & 15);
        unsigned long long packed[S];
        pack_digits8<S>(y, W, packed);
#pragma unroll
        for (int t = 0; t < S; ++t) *reinterpret_cast<unsigned long long*>(digits + t * plane + off) = packed[t];
    }
}

// One wave per padded row: row scale and `slices` digit planes of X_n.
template <int S>
__global__ __launch_bounds__(256) void k_encode_int8(const double* __restrict__ buf0,
                                                     const double* __restrict__ buf1, int ld,
                                                     const State* __restrict__ st,
                                                     int8_t* __restrict__ digits,
                                                     double* __restrict__ scale) {
    if (st->done || st->phase != 1) return;
    encode_row<S>(st->cur ? buf1 : buf0, ld, blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63, digits, scale,
                  0, ld);
}

// One workgroup per padded row, the row held in registers between the max and
// the digit pass (one HBM read of X instead of two).  Thread t takes columns
// 8 t + 2048 c .. +8 for c < CH, so rows up to 2048 CH columns fit.  Blocks
// are mapped to rows XCD-contiguously (block b runs on XCD b % 8 and takes
// row (b % 8) ld / 8 + b / 8), so the four rows whose 32-byte pieces share a
// 128-byte line of a digit block are written through one L2 at nearly the
// same time.  Same digits as encode_row (the row maximum is order-free).
constexpr int ENC_CH = 8;

template <int S>
__global__ __launch_bounds__(256) void k_encode_int8_reg(const double* __restrict__ buf0,
                                                         const double* __restrict__ buf1, int ld,
                                                         const State* __restrict__ st,
                                                         int8_t* __restrict__ digits,
                                                         double* __restrict__ scale) {
    if (st->done || st->phase != 1) return;
    const double* __restrict__ X = st->cur ? buf1 : buf0;
    const int b = blockIdx.x;
    const int i = (b & 7) * (ld >> 3) + (b >> 3);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double* row = X + (size_t)i * ld;
    double4 va[ENC_CH], vb[ENC_CH];
    double m = 0.0;
#pragma unroll
    for (int c = 0; c < ENC_CH; ++c) {
        const int j = 8 * tid + 2048 * c;
        if (j < ld) {
            va[c] = *reinterpret_cast<const double4*>(row + j);
            vb[c] = *reinterpret_cast<const double4*>(row + j + 4);
            m = fmax(m, fmax(fmax(fabs(va[c].x), fabs(va[c].y)), fmax(fabs(va[c].z), fabs(va[c].w))));
            m = fmax(m, fmax(fmax(fabs(vb[c].x), fabs(vb[c].y)), fmax(fabs(vb[c].z), fabs(vb[c].w))));
        }
    }
    m = wred_max(m);
    __shared__ double wm[4];
    if (lane == 0) wm[w] = m;
    __syncthreads();
    m = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
    double sc;
    const double inv = row_scale(m, &sc);
    if (tid == 0) scale[i] = sc;
    const size_t plane = (size_t)ld * ld;
    const size_t rowblk = (size_t)(i >> 5) * (ld >> 5);
    const int r32 = i & 31;
#pragma unroll
    for (int c = 0; c < ENC_CH; ++c) {
        const int j = 8 * tid + 2048 * c;
        if (j < ld) {
            double y[8] = {va[c].x * inv, va[c].y * inv, va[c].z * inv, va[c].w * inv,
                           vb[c].x * inv, vb[c].y * inv, vb[c].z * inv, vb[c].w * inv};
            const size_t off = (rowblk + (j >> 5)) * 1024 + r32 * 32 + 16 * (((j >> 4) & 1) ^ dswz(r32)) + (j & 15);
            unsigned long long packed[S];
            pack_digits8<S>(y, digit_bits(ld, S), packed);
#pragma unroll
            for (int t = 0; t < S; ++t) *reinterpret_cast<unsigned long long*>(digits + t * plane + off) = packed[t];
        }
    }
}

// Upper-triangle encode.  When the products write only their upper tiles
// (upper-only mode), X_n is valid on and above the diagonal and rmax[i]
// holds max_j |X_ij| as a bit pattern (accumulated by the product that wrote
// X_n).  One workgroup per 32 x 32 block (I, J), I <= J: the block is read
// once and written as digit block (I, J) with the scales of rows I and, read
// back transposed from LDS, as digit block (J, I) with the scales of rows J.
// Same digits as encode_row (same scale, same per-element arithmetic).  The
// diagonal blocks also write the row scales and clear rmax_next, which the
// next product fills.
__device__ __forceinline__ void pack_digits4(const double (&x)[4], double inv, int S, int W, int8_t* __restrict__ out,
                                             size_t plane) {
    double y[4] = {x[0] * inv, x[1] * inv, x[2] * inv, x[3] * inv};
    if (W == 8) {
        unsigned long long u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) u[q] = excess_digits(y[q], S);
        for (int t = 0; t < S; ++t) {
            uint32_t packed = 0u;
#pragma unroll
            for (int q = 0; q < 4; ++q) packed |= excess_digit(u[q], S, t) << (8 * q);
            *reinterpret_cast<uint32_t*>(out + t * plane) = packed;
        }
        return;
    }
    for (int t = 0; t < S; ++t) {
        const double wt = ldexp(1.0, 6 + 7 * t);
        const double iw = ldexp(1.0, -(6 + 7 * t));
        uint32_t packed = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double d = rint(y[q] * wt);
            y[q] -= d * iw;
            packed |= (uint32_t)(uint8_t)(int8_t)d << (8 * q);
        }
        *reinterpret_cast<uint32_t*>(out + t * plane) = packed;
    }
}

__device__ __forceinline__ double scale_inv(unsigned long long bits, double* s_out) {
    return row_scale(__longlong_as_double((long long)bits), s_out);
}

template <int S>
__global__ __launch_bounds__(256) void k_encode_int8_upper(const double* __restrict__ buf0,
                                                           const double* __restrict__ buf1, int ld,
                                                           const State* __restrict__ st,
                                                           int8_t* __restrict__ digits,
                                                           double* __restrict__ scale,
                                                           unsigned long long* __restrict__ rmax) {
    if (st->done || st->phase != 1) return;
    const double* __restrict__ X = st->cur ? buf1 : buf0;
    const unsigned long long* __restrict__ rm = rmax + (size_t)st->cur * ld;
    unsigned long long* __restrict__ rm_next = rmax + (size_t)(1 - st->cur) * ld;
    const int nb = ld >> 5;
    // block (I, J) of the upper triangle, row-major over I
    const int t = blockIdx.x;
    int I = (int)((2.0 * nb + 1.0 - sqrt((2.0 * nb + 1.0) * (2.0 * nb + 1.0) - 8.0 * (double)t)) / 2.0);
    I = max(0, min(I, nb - 1));
    while (I > 0 && I * nb - I * (I - 1) / 2 > t) --I;
    while (I + 1 < nb && (I + 1) * nb - (I + 1) * I / 2 <= t) ++I;
    const int J = I + (t - (I * nb - I * (I - 1) / 2));
    const int tid = threadIdx.x;
    const int r = tid >> 3, c0 = (tid & 7) * 4;
    const size_t plane = (size_t)ld * ld;
    const double4 v = *reinterpret_cast<const double4*>(X + (size_t)(I * 32 + r) * ld + J * 32 + c0);
    const double x[4] = {v.x, v.y, v.z, v.w};
    double sc;
    const double inv = scale_inv(rm[I * 32 + r], &sc);
    pack_digits4(x, inv, S, digit_bits(ld, S), digits + ((size_t)I * nb + J) * 1024 + r * 32 + 16 * ((c0 >> 4) ^ dswz(r)) + (c0 & 15),
                 plane);
    if (I == J) {
        if ((tid & 7) == 0) {
            scale[I * 32 + r] = sc;
            rm_next[I * 32 + r] = 0ull;
        }
        return;
    }
    __shared__ double T[32][33];
    T[r][c0] = x[0];
    T[r][c0 + 1] = x[1];
    T[r][c0 + 2] = x[2];
    T[r][c0 + 3] = x[3];
    __syncthreads();
    // row J*32 + r of X, columns I*32 + c0 .. + 3 = column r of the block, rows c0 ..
    const double xt[4] = {T[c0][r], T[c0 + 1][r], T[c0 + 2][r], T[c0 + 3][r]};
    const double invt = scale_inv(rm[J * 32 + r], nullptr);
    pack_digits4(xt, invt, S, digit_bits(ld, S), digits + ((size_t)J * nb + I) * 1024 + r * 32 + 16 * ((c0 >> 4) ^ dswz(r)) + (c0 & 15),
                 plane);
}

// Grouped: work item = 4 rows of one system; fixed grid, grid-stride loop.
template <int S>
__global__ __launch_bounds__(256) void k_encode_int8_grouped(const GroupDesc* __restrict__ g) {
    const int total = g->total_rowq;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int s = group_find(g->row_off, g->nsys, item);
        const SysView& v = g->sys[s];
        const State* st = v.st;
        if (st->done || st->phase != 1) continue;
        const int i = (item - g->row_off[s]) * 4 + (threadIdx.x >> 6);
        encode_row<S>(st->cur ? v.buf1 : v.buf0, v.ld, i, threadIdx.x & 63, v.digits, v.scale, 0, v.ld);
    }
}

// ------------------------------------------------------------------ product
// One 512-thread workgroup per upper-triangular 128 x 128 tile; wave w
// covers rows 32 (w >> 1) .. +32 and columns 64 (w & 1) .. +64 as two 32 x 32
// blocks of v_mfma_i32_32x32x32_i8 per level (NL x 2 accumulators of 16
// int32).  Each K stage stages 2 operands x S planes x 4 row blocks x KS
// k blocks of 1 KiB through an LDS ring in the blocked layout, filled by
// global -> LDS loads one stage ahead of the products.
constexpr int QB = 128;          // tile
constexpr int QK = 32;           // k bytes per block

// K stage: KS blocks of 32 k-bytes; ring depth NST.  Configuration C = 0
// (the default): up to five planes fit a 64-byte stage twice in LDS
// (2 x 80 KiB at five), which halves the barriers per product against
// 32-byte stages; six planes keep 32-byte stages three deep (3 x 48 KiB).
// C = 1: 32-byte stages three deep; C = 2: 32-byte stages four deep (up to
// five planes).  The autotuner picks C per size for dense products.
template <int S, int C = 0> struct I8Stage {
    static constexpr int KS = (C == 0 && S <= 5) ? 2 : 1;
    static constexpr int NST = C == 0 ? (S <= 5 ? 2 : 3) : (C == 1 ? 3 : 4);
    static_assert(NST * 2 * S * 4 * KS <= 160, "stage ring exceeds the LDS");
};
// Configurations valid for S planes.
__host__ __device__ constexpr bool i8_cfg_ok(int S, int C) { return C == 0 || C == 1 || (C == 2 && S <= 5); }

// The staging ring; after the K loop the same LDS holds half of the finished
// tile, transposed, so the mirrored (lower-triangle) copy is written as
// whole rows instead of one 8-byte element per row.  Row stride 129 doubles
// spreads the column-wise LDS stores over the banks.
constexpr int TR_LD = 129;

template <int S, int C = 0>
struct I8Smem {
    union {
        int8_t buf[I8Stage<S, C>::NST][2 * S * 4 * I8Stage<S, C>::KS][1024];   // [stage][((op S + slice) 4 + row block) KS + k block][block]
        double tr[64][TR_LD];                  // [tile column (one half)][tile row]
        struct {
            double xs[128][128];                   // the X_n tile (upper-only mode), staged for the update
            unsigned long long rm[128], cm[128];   // tile row / column maxima (upper-only mode)
            double red[3][8];                      // per-wave partials, after the last use of tr / rm / cm
        } mx;
    };
};

// One 128 x 128 output tile (bi, bj) of one system; all 512 threads of the
// workgroup take part (the body contains barriers).  kmode 0: the whole
// tile; kmode 1: only K stages [kc0, kc1), whose int32 level accumulators are
// stored to chunk_acc (one chunk of a tile split along K); kmode 2: no K
// loop, the accumulators are the sum of the nchunks chunks at chunk_acc (the
// integer sums are exact, so a split tile equals an unsplit one), then the
// epilogue.  Chunk layout: int4 [NL][2][4][512 threads] (accumulator elements
// 4q .. 4q + 3 of level L, column block c), so that each wave moves 1 KiB
// per instruction.  UPPER: write the tile
// only (no mirrored copy below the diagonal) and fold its row and column
// maxima of |X_{n+1}| into rmax_next (bit patterns of non-negative doubles
// order like the values, so atomicMax on them is exact and order-free).
template <int S, int NL, bool THR, bool UPPER, int C = 0>
__device__ __forceinline__ void int8x_tile(double* __restrict__ buf0, double* __restrict__ buf1, int ld,
                           const State* __restrict__ st, const int8_t* __restrict__ digits,
                           const double* __restrict__ scale, double* __restrict__ part, int bi, int bj,
                           I8Smem<S, C>& sm, const int* __restrict__ env,
                           unsigned long long* __restrict__ rmax_next, int kmode = 0, int kc0 = 0,
                           int kc1 = -1, int* __restrict__ chunk_acc = nullptr, int nchunks = 0) {
    const int nt = ld / QB;
    const int t = tri_index(bi, bj, nt);
    const int i0 = bi * QB, j0 = bj * QB;
    const double* __restrict__ Xc = st->cur ? buf1 : buf0;
    double* __restrict__ Xn = st->cur ? buf0 : buf1;
    const size_t plane = (size_t)ld * ld;
    const int nb = ld >> 5;          // blocks per block row

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;

    constexpr int KS = I8Stage<S, C>::KS, NST = I8Stage<S, C>::NST;
    constexpr int NBLK = 2 * S * 4 * KS;        // 1 KiB blocks per stage
    constexpr int PER = NBLK * 64 / 512;        // 16-byte chunks per thread
    static_assert((NBLK * 64) % 512 == 0, "stage must split evenly over 512 threads");

    static_assert(NL == S || NL == S + 1, "levels: the triangle or one more");
    v16i acc[NL][2];
#pragma unroll
    for (int L = 0; L < NL; ++L)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[L][c][r] = 0;

    // fragment address inside a block: row lane % 32, k-half lane / 32
    const int fr = lane & 31;
    const int foff = fr * 32 + 16 * ((lane >> 5) ^ dswz(fr));
    // K stages: all of them (or chunk [kc0, kc1)), or for a thresholded X
    // those holding a 32-column block set in both panels' block masks (the
    // other stages multiply a zero block on one side)
    int ks = 0, nk = ld / (QK * KS);
    if (kc1 >= 0) {
        ks = kc0;
        nk = kc1;
    }
    const int nbk = ld / QK;
    bool holes = false;
    const unsigned long long* mk = THR ? env_mask(env, nt) : nullptr;
    const unsigned long long* mi = THR ? mk + (size_t)bi * mask_words(ld) : nullptr;
    const unsigned long long* mj = THR ? mk + (size_t)bj * mask_words(ld) : nullptr;
    if (THR) {
        // the stages between the first and the last common block; when some
        // stage in between has none (the blocks are scattered, not banded),
        // the loop below visits the working stages only
        const unsigned long long mword = common_mask_word(mi, mj, nbk);
        // per lane: stages of its word holding a common block (KS divides
        // 64, so no stage straddles two words) and its last common block;
        // then the wave's sum and maximum
        int stages = 0, b1 = -1;
        if (mword) {
            unsigned long long m = mword;
            if (KS == 2) m = (m | (m >> 1)) & 0x5555555555555555ull;
            stages = __popcll(m);
            b1 = (lane << 6) + 63 - __builtin_clzll(mword);
        }
        for (int o = 32; o > 0; o >>= 1) {
            stages += __shfl_xor(stages, o, 64);
            b1 = max(b1, __shfl_xor(b1, o, 64));
        }
        if (b1 < 0) {
            ks = nk = 0;
        } else {
            ks = next_block_in_wave(mword, 0, nbk) / KS;
            nk = b1 / KS + 1;
            holes = stages < nk - ks;
        }
    }

    // Fragment reads are written in order of first use (B plane 0, the A
    // planes, B planes 1 ..), the products in level order, and the scheduler
    // is held to a pattern of one read per two products that keeps every
    // read LA product pairs ahead of its first use, so a stage starts after
    // 3 + LA reads instead of the whole set.
    auto compute = [&](int stg) {
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            auto rdA = [&](int sl) {
                return *reinterpret_cast<const v4i*>(&sm.buf[stg][(sl * 4 + wr) * KS + kk][foff]);
            };
            auto rdB = [&](int uu, int c) {
                return *reinterpret_cast<const v4i*>(&sm.buf[stg][(S * 4 + uu * 4 + wc * 2 + c) * KS + kk][foff]);
            };
            v4i a[S], b[S][2];
            b[0][0] = rdB(0, 0);
            b[0][1] = rdB(0, 1);
#pragma unroll
            for (int tt = 0; tt < S; ++tt) a[tt] = rdA(tt);
#pragma unroll
            for (int uu = 1; uu < S; ++uu) {
                b[uu][0] = rdB(uu, 0);
                b[uu][1] = rdB(uu, 1);
            }
            // level tt + uu accumulates a[tt] b[uu]
#pragma unroll
            for (int uu = 0; uu < S; ++uu)
#pragma unroll
                for (int tt = 0; tt < S && tt < NL - uu; ++tt)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        acc[tt + uu][c] =
                            __builtin_amdgcn_mfma_i32_32x32x32_i8(a[tt], b[uu][c], acc[tt + uu][c], 0, 0, 0);
        }
        constexpr int LA = 2;                                  // lookahead in reads
        constexpr int R = 3 * S * KS, P = (S * (S + 1) / 2 + (NL - S) * (S - 1)) * KS;   // reads, product pairs
        constexpr int MID = R - 3 - LA;
        __builtin_amdgcn_sched_group_barrier(0x100, 3 + LA, 0);
#pragma unroll
        for (int q = 0; q < MID; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 2 * (P - MID), 0);
    };
    // Global -> LDS loads without register staging: wave w moves blocks w,
    // w + 8, ... of a stage, one 1 KiB block per instruction (16 bytes per
    // lane).  Stage kt + NST - 1 is issued while stage kt is multiplied;
    // before reading stage kt a wave waits for its own loads of stage kt (at
    // most the PER loads of stage kt + 1 stay outstanding in a three-deep
    // ring), and a barrier then makes every wave's blocks visible.
    auto issue = [&](int kb, int stg) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int blk = w + 8 * m;
            const int kk = blk % KS, ob = blk / KS;
            const int op = ob / (S * 4);
            const int rem = ob - op * (S * 4);
            const int sl = rem >> 2, rb = rem & 3;
            const int grb = ((op ? j0 : i0) >> 5) + rb;
            const int8_t* g = digits + sl * plane + ((size_t)grb * nb + kb * KS + kk) * 1024 + 16 * lane;
            __builtin_amdgcn_global_load_lds((const void*)g,
                                             (__attribute__((address_space(3))) void*)&sm.buf[stg][blk][0], 16, 0, 0);
        }
    };
    if (kmode == 2) nk = ks;          // accumulators come from the chunks
    if (!holes) {
        // every stage of [ks, nk) works: a plain loop
        for (int q = 0; q < NST - 1; ++q)
            if (ks + q < nk) issue(ks + q, q);
        for (int kt = ks; kt < nk; ++kt) {
            // this wave's blocks of stage kt have landed in LDS once only
            // stage kt + 1's loads (three-deep ring) or none (two-deep) are
            // outstanding; the bare barrier (no fence, which would wait for
            // every outstanding load) then covers the other waves' blocks, and
            // every wave has finished reading the buffer that stage
            // kt + NST - 1 overwrites
            if (NST == 4 && kt + 2 < nk) __builtin_amdgcn_s_waitcnt(0x0F70 | (2 * PER));   // vmcnt(2 PER)
            else if (NST >= 3 && kt + 1 < nk) __builtin_amdgcn_s_waitcnt(0x0F70 | PER);   // vmcnt(PER)
            else __builtin_amdgcn_s_waitcnt(0x0F70);                                      // vmcnt(0)
            __builtin_amdgcn_s_barrier();
            if (kt + NST - 1 < nk) issue(kt + NST - 1, (kt + NST - 1 - ks) % NST);
            compute((kt - ks) % NST);
        }
    }
    // with holes: the working stages in increasing order go round the ring:
    // ic is the next stage to issue, n_iss / n_done count stages issued /
    // multiplied (the common mask is reloaded here, so that it is not live
    // across the plain loop)
    const unsigned long long mword = (THR && holes) ? common_mask_word(mi, mj, nbk) : 0ull;
    auto next_stage = [&](int s) -> int {      // first working stage >= s, or nk
        const int b = next_block_in_wave(mword, s * KS, nbk);
        return b >= nbk ? nk : b / KS;
    };
    int ic = holes ? next_stage(ks) : nk, n_iss = 0, n_done = 0;
    while (n_iss < NST - 1 && ic < nk) {
        issue(ic, n_iss % NST);
        ++n_iss;
        ic = next_stage(ic + 1);
    }
    while (n_done < n_iss) {
        // this wave's blocks of the stage in ring slot n_done have landed in
        // LDS once only the next stage's loads (three-deep ring) or none
        // (two-deep) are outstanding; the bare barrier (no fence, which would
        // wait for every outstanding load) then covers the other waves'
        // blocks, and every wave has finished reading the slot that the next
        // issue overwrites
        if (NST == 4 && n_iss - n_done == 3) __builtin_amdgcn_s_waitcnt(0x0F70 | (2 * PER));   // vmcnt(2 PER)
        else if (NST >= 3 && n_iss - n_done >= 2) __builtin_amdgcn_s_waitcnt(0x0F70 | PER);   // vmcnt(PER)
        else __builtin_amdgcn_s_waitcnt(0x0F70);                                              // vmcnt(0)
        __builtin_amdgcn_s_barrier();
        if (ic < nk) {
            issue(ic, n_iss % NST);
            ++n_iss;
            ic = next_stage(ic + 1);
        }
        compute(n_done % NST);
        ++n_done;
    }
    __syncthreads();
    constexpr int CH = NL * 2 * 16 * 512;   // int32 per chunk
    if (kmode == 1) {
        int4* out = reinterpret_cast<int4*>(chunk_acc);
#pragma unroll
        for (int L = 0; L < NL; ++L)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    out[((L * 2 + c) * 4 + q) * 512 + tid] =
                        make_int4(acc[L][c][4 * q], acc[L][c][4 * q + 1], acc[L][c][4 * q + 2], acc[L][c][4 * q + 3]);
        return;
    }
    if (kmode == 2) {
        for (int ch = 0; ch < nchunks; ++ch) {
            const int4* in = reinterpret_cast<const int4*>(chunk_acc + (size_t)ch * CH);
#pragma unroll
            for (int L = 0; L < NL; ++L)
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int4 v = in[((L * 2 + c) * 4 + q) * 512 + tid];
                        acc[L][c][4 * q] += v.x;
                        acc[L][c][4 * q + 1] += v.y;
                        acc[L][c][4 * q + 2] += v.z;
                        acc[L][c][4 * q + 3] += v.w;
                    }
        }
    }

    if constexpr (UPPER) {
        // the X_n tile to LDS in one burst (16 rows of 1 KiB per wave, all in
        // flight at once) instead of dependent global loads inside the
        // update; the ring is free once every wave is past its last stage
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int row = w + 8 * m;
            __builtin_amdgcn_global_load_lds((const void*)(Xc + (size_t)(i0 + row) * ld + j0 + 2 * lane),
                                             (__attribute__((address_space(3))) void*)&sm.mx.xs[row][0], 16, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        __syncthreads();
    }
    // epilogue: combine levels in FP64, apply the SP2 update, partials.
    // Partial sums are kept per column block c in row order and added at the
    // end, the same order in both layouts (so both give identical partials).
    const int br = st->branch;
    const bool mirror = bi != bj;
    const int W = digit_bits(ld, S), E2 = 2 * digit_e0(W);
    double trc[2] = {0.0, 0.0}, froc[2] = {0.0, 0.0}, idmc[2] = {0.0, 0.0};
    auto element = [&](int c, int r, int gi, int gj, double sj) -> double {
        double v = 0.0;
#pragma unroll
        for (int L = NL - 1; L >= 0; --L) v += ldexp((double)acc[L][c][r], -(E2 + W * L));
        // s_i s_j first: the product is then the same for (i, j) and (j, i)
        // (the diagonal tiles form both), so X stays exactly symmetric
        const double p = v * (scale[gi] * sj);
        const double x = UPPER ? sm.mx.xs[gi - i0][gj - j0] : Xc[(size_t)gi * ld + gj];
        const double xn = br ? 2.0 * x - p : p;
        Xn[(size_t)gi * ld + gj] = xn;
        if (gi == gj) trc[c] += xn;
        froc[c] += xn * xn;
        idmc[c] += (p - x) * (p - x);
        return xn;
    };
    // v_mfma_i32_32x32x32_i8 result: lane l, element r is row 8 (r/4) + 4 (l/32) + r%4, column l%32
    auto row_of = [&](int r) { return i0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); };
    if (UPPER) {
        // tile row and column maxima are combined in LDS, then one global
        // atomic per row (and per column off the diagonal) of the tile
        if (tid < 128) sm.mx.rm[tid] = 0ull;
        else if (tid < 256) sm.mx.cm[tid - 128] = 0ull;
        __syncthreads();
        const int gj0 = j0 + wc * 64 + (lane & 31), gj1 = gj0 + 32;
        const double sj0 = scale[gj0], sj1 = scale[gj1];
        double cmx0 = 0.0, cmx1 = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int gi = row_of(r);
            const double a = fabs(element(0, r, gi, gj0, sj0));
            const double b = fabs(element(1, r, gi, gj1, sj1));
            cmx0 = fmax(cmx0, a);
            cmx1 = fmax(cmx1, b);
            // row maximum over the wave's 64 columns (32 lanes of this half)
            double m = fmax(a, b);
            for (int o = 16; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
            if ((lane & 31) == 0) atomicMax(&sm.mx.rm[gi - i0], (unsigned long long)__double_as_longlong(m));
        }
        if (mirror) {
            // column maxima over the wave's 32 rows: row maxima of rows gj over
            // these columns of their lower part (a diagonal tile is symmetric)
            cmx0 = fmax(cmx0, __shfl_xor(cmx0, 32, 64));
            cmx1 = fmax(cmx1, __shfl_xor(cmx1, 32, 64));
            if (lane < 32) {
                atomicMax(&sm.mx.cm[gj0 - j0], (unsigned long long)__double_as_longlong(cmx0));
                atomicMax(&sm.mx.cm[gj1 - j0], (unsigned long long)__double_as_longlong(cmx1));
            }
        }
        __syncthreads();
        if (tid < 128) atomicMax(rmax_next + i0 + tid, sm.mx.rm[tid]);
        else if (mirror && tid < 256) atomicMax(rmax_next + j0 + tid - 128, sm.mx.cm[tid - 128]);
    } else {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int gj = j0 + wc * 64 + c * 32 + (lane & 31);
            const double sj = scale[gj];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int gi = row_of(r);
                const double xn = element(c, r, gi, gj, sj);
                if (mirror) sm.tr[wc * 32 + (lane & 31)][gi - i0] = xn;
            }
            if (mirror) {
                // columns j0 + 64 wc' + 32 c + (0..31) of every wave: 64 rows of
                // the mirrored block, 128 doubles each, written one half row per
                // wave and instruction
                __syncthreads();
#pragma unroll 4
                for (int q = 0; q < 16; ++q) {
                    const int rh = w + 8 * q;
                    const int jj = rh >> 1, col = (rh & 1) * 64 + lane;
                    const int gr = j0 + (jj >> 5) * 64 + c * 32 + (jj & 31);
                    Xn[(size_t)gr * ld + i0 + col] = sm.tr[jj][col];
                }
                __syncthreads();
            }
        }
    }
    double tr = trc[0] + trc[1], fro = froc[0] + froc[1], idm = idmc[0] + idmc[1];
    tr = wred_sum(tr);
    fro = wred_sum(fro);
    idm = wred_sum(idm);
    double (*red)[8] = sm.mx.red;
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

// Workgroups [0, t_full): whole tiles at visiting positions [0, t_full),
// dealt over the XCDs.  Workgroups from t_full on: the tiles at positions
// t_full, t_full + 1, ... (the last, partly filled wave of a launch), each
// split into nsplit chunks of the K loop whose accumulators go to chunk_acc;
// k_gemm_int8x_tail finishes them.
//
// THR: tiles are visited diagonal by diagonal (bj - bi = 0, 1, ..), so the
// tiles of a banded X, the only ones with a K range, are the first ones
// dispatched and spread over every CU (the XCD-dealt super-tile order would
// put most of them on the XCDs that take the short rows near the end of the
// triangle); tile_group does not apply.
// Tile at position pos of the diagonal-major order of the upper triangle of
// nt x nt tiles: diagonal d starts at d nt - d (d - 1) / 2.
__device__ __forceinline__ void diag_tile(int pos, int nt, int& bi, int& bj) {
    const double b = 2.0 * nt + 1.0;
    int d = (int)((b - sqrt(b * b - 8.0 * pos)) * 0.5);
    auto start = [nt](int e) { return e * nt - e * (e - 1) / 2; };
    while (d > 0 && start(d) > pos) --d;
    while (d + 1 < nt && start(d + 1) <= pos) ++d;
    bi = pos - start(d);
    bj = bi + d;
}

template <int S, int NL, bool THR, bool UPPER, int C = 0>
__global__ __launch_bounds__(512) void k_gemm_int8x(double* __restrict__ buf0, double* __restrict__ buf1,
                                                    int ld, const State* __restrict__ st,
                                                    const int8_t* __restrict__ digits,
                                                    const double* __restrict__ scale,
                                                    double* __restrict__ part, const int* __restrict__ env,
                                                    unsigned long long* __restrict__ rmax, int tile_group,
                                                    int t_full, int nsplit, int* __restrict__ chunk_acc,
                                                    int when_full) {
    if (st->done || st->phase != 1 || (when_full && !st->full_fill)) return;
    extern __shared__ __align__(16) int8_t smem_raw[];
    I8Smem<S, C>& sm = *reinterpret_cast<I8Smem<S, C>*>(smem_raw);
    const int nt = ld / QB, w = blockIdx.x;
    int pos, kmode = 0, kc0 = 0, kc1 = -1;
    int* cacc = nullptr;
    if (THR) {
        pos = w;
    } else if (w < t_full) {
        pos = xcd_deal(w, t_full);
    } else {
        const int j = w - t_full, p = j / nsplit, ch = j - p * nsplit, nk = ld / (QK * I8Stage<S, C>::KS);
        pos = t_full + p;
        kmode = 1;
        kc0 = ch * nk / nsplit;
        kc1 = (ch + 1) * nk / nsplit;
        cacc = chunk_acc + (size_t)j * (NL * 2 * 16 * 512);
    }
    int bi, bj;
    if (THR) diag_tile(pos, nt, bi, bj);
    else order_tile(pos, nt, tile_group, bi, bj);
    int8x_tile<S, NL, THR, UPPER, C>(buf0, buf1, ld, st, digits, scale, part, bi, bj, sm, env,
                              UPPER ? rmax + (size_t)(1 - st->cur) * ld : nullptr, kmode, kc0, kc1, cacc, 0);
}

// order_tile with one step per super-tile row instead of one per super-tile
// (the list kernel maps every tile of the triangle): the same tile for
// every position.
__device__ __forceinline__ void order_tile_rows(int t, int nt, int G, int& bi, int& bj) {
    if (G <= 0 || G > nt) G = nt;
    int I = 0, gi = min(G, nt);
    for (;;) {
        gi = min(G, nt - I * G);
        const int row = gi * (gi + 1) / 2 + gi * (nt - I * G - gi);
        if (t < row || I * G + gi >= nt) break;
        t -= row;
        ++I;
    }
    const int d = gi * (gi + 1) / 2;
    if (t < d) {
        int li = 0, off = 0;
        while (t >= off + (gi - li)) { off += gi - li; ++li; }
        bi = I * G + li;
        bj = I * G + li + (t - off);
        return;
    }
    t -= d;
    const int J = I + 1 + t / (gi * G);
    t -= (J - I - 1) * gi * G;
    const int gj = min(G, nt - J * G);
    bi = I * G + t / gj;
    bj = J * G + t % gj;
}

// ---- thresholded products driven by a work list (int8 from the first product on)
//
// Zero-tile flags tz (one row of T upper tiles per X buffer, kept with the
// threshold pass): a tile whose K range is empty and whose X_n tile is all
// zero has X_{n+1} = 0 there under either branch.  k_tile_list visits the
// tiles in the product's G x G super-tile order; such a tile gets zero
// partials and is left out when its destination tile is already all zero,
// or is listed for plain zero stores (no reads) when it is not; every other
// tile is listed for the product.  The list holds (zero_store << 30) |
// (bi << 15) | bj; list_ctr[0] counts entries, list_ctr[1] hands them out in
// list order, so whatever the order the work is balanced, and concurrent
// workgroups work on nearby tiles that share row panels.
__global__ void k_list_reset(int* __restrict__ list_ctr, const State* __restrict__ st) {
    if (st->done || st->phase != 1 || st->full_fill) return;
    if (threadIdx.x < 2) list_ctr[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_tile_list(const State* __restrict__ st, const int* __restrict__ env,
                                                   const int* __restrict__ tz, int nt, int tile_group,
                                                   double* __restrict__ part, int* __restrict__ list,
                                                   int* __restrict__ list_ctr) {
    if (st->done || st->phase != 1 || st->full_fill) return;
    const int T = nt * (nt + 1) / 2;
    const int pos = blockIdx.x * 256 + threadIdx.x;
    bool listed = false;
    int item = 0;
    if (pos < T) {
        int bi, bj;
        order_tile_rows(pos, nt, tile_group, bi, bj);
        const int t = tri_index(bi, bj, nt);
        // no 32-column block set in both panels' masks: the product tile is zero
        const unsigned long long* mk = env_mask(env, nt);
        const int W = mask_words(nt * QB), nbk = nt * QB / QK;
        const bool k_empty = next_common_block(mk + (size_t)bi * W, mk + (size_t)bj * W, 0, nbk) >= nbk;
        const bool zero_next = k_empty && tz[(size_t)st->cur * T + t] != 0;
        if (zero_next && tz[(size_t)(1 - st->cur) * T + t] != 0) {
            part[3 * t + 0] = 0.0;
            part[3 * t + 1] = 0.0;
            part[3 * t + 2] = 0.0;
        } else {
            listed = true;
            item = ((zero_next ? 1 : 0) << 30) | (bi << 15) | bj;
        }
    }
    // one atomic per wave
    const unsigned long long m = __ballot(listed);
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == 0 && m) base = atomicAdd(&list_ctr[0], __popcll(m));
    base = __shfl(base, 0, 64);
    if (listed) list[base + __popcll(m & ((1ull << lane) - 1ull))] = item;
}

// One workgroup per CU takes list entries until none is left (every
// workgroup leaves once the shared counter passes the entry count).
template <int S, int NL>
__global__ __launch_bounds__(512) void k_gemm_int8x_list(double* __restrict__ buf0, double* __restrict__ buf1,
                                                         int ld, const State* __restrict__ st,
                                                         const int8_t* __restrict__ digits,
                                                         const double* __restrict__ scale,
                                                         double* __restrict__ part, const int* __restrict__ env,
                                                         int* __restrict__ tz, const int* __restrict__ list,
                                                         int* __restrict__ list_ctr) {
    if (st->done || st->phase != 1 || st->full_fill) return;
    extern __shared__ __align__(16) int8_t smem_raw[];
    I8Smem<S>& sm = *reinterpret_cast<I8Smem<S>*>(smem_raw);
    // the entry index is passed through the first word of the staging ring,
    // which no tile uses between the barriers around it (the ring fills the
    // 160 KiB of LDS; a separate shared variable would not fit)
    volatile int& s_k = *reinterpret_cast<int*>(smem_raw);
    const int nt = ld / QB, T = nt * (nt + 1) / 2;
    const int n = list_ctr[0];
    int* __restrict__ tzn = tz + (size_t)(1 - st->cur) * T;
    double* __restrict__ Xn = st->cur ? buf0 : buf1;
    for (;;) {
        if (threadIdx.x == 0) s_k = atomicAdd(&list_ctr[1], 1);
        __syncthreads();
        const int k = s_k;
        __syncthreads();
        if (k >= n) break;
        const int it = list[k];
        const int bi = (it >> 15) & 0x7fff, bj = it & 0x7fff;
        const int t = tri_index(bi, bj, nt);
        if (it >> 30) {
            const double2 z = make_double2(0.0, 0.0);
            for (int e = threadIdx.x; e < QB * QB / 2; e += 512) {
                const int r = e / (QB / 2), c = 2 * (e % (QB / 2));
                *reinterpret_cast<double2*>(Xn + (size_t)(bi * QB + r) * ld + bj * QB + c) = z;
                if (bi != bj) *reinterpret_cast<double2*>(Xn + (size_t)(bj * QB + r) * ld + bi * QB + c) = z;
            }
            if (threadIdx.x == 0) {
                part[3 * t + 0] = 0.0;
                part[3 * t + 1] = 0.0;
                part[3 * t + 2] = 0.0;
                tzn[t] = 1;
            }
        } else {
            int8x_tile<S, NL, true, false>(buf0, buf1, ld, st, digits, scale, part, bi, bj, sm, env, nullptr);
            if (threadIdx.x == 0) tzn[t] = 0;
        }
        __syncthreads();
    }
}

// Epilogue of the split tiles: workgroup p takes the summed chunks of the
// tile at visiting position t_full + p and applies the update.
template <int S, int NL, bool UPPER, int C = 0>
__global__ __launch_bounds__(512) void k_gemm_int8x_tail(double* __restrict__ buf0, double* __restrict__ buf1,
                                                         int ld, const State* __restrict__ st,
                                                         const int8_t* __restrict__ digits,
                                                         const double* __restrict__ scale,
                                                         double* __restrict__ part,
                                                         unsigned long long* __restrict__ rmax, int tile_group,
                                                         int t_full, int nsplit, int* __restrict__ chunk_acc,
                                                         int when_full) {
    if (st->done || st->phase != 1 || (when_full && !st->full_fill)) return;
    extern __shared__ __align__(16) int8_t smem_raw[];
    I8Smem<S, C>& sm = *reinterpret_cast<I8Smem<S, C>*>(smem_raw);
    int bi, bj;
    order_tile(t_full + blockIdx.x, ld / QB, tile_group, bi, bj);
    // k_chunk_sum has added the tile's chunks into its first one
    int8x_tile<S, NL, false, UPPER, C>(buf0, buf1, ld, st, digits, scale, part, bi, bj, sm, nullptr,
                                    UPPER ? rmax + (size_t)(1 - st->cur) * ld : nullptr, 2, 0, -1,
                                    chunk_acc + (size_t)blockIdx.x * nsplit * (NL * 2 * 16 * 512), 1);
}

// The int32 accumulators of the nsplit K chunks of each split tile, added
// into the tile's first chunk (exact: every partial sum over a range of K is
// bounded like the whole sum).  kChunkSumParts workgroups per tile, each over
// an equal share of the tile's NL x 2 x 16 x 512 accumulators, so the sums
// are read by many CUs at once instead of by the tile's one tail workgroup.
constexpr int kChunkSumParts = 8;
template <int NL>
__global__ __launch_bounds__(256) void k_chunk_sum(int* __restrict__ chunk_acc, int nsplit,
                                                   const State* __restrict__ st, int when_full) {
    if (st->done || st->phase != 1 || (when_full && !st->full_fill)) return;
    constexpr int CH4 = NL * 2 * 16 * 512 / 4;          // int4 per chunk
    constexpr int PER = CH4 / kChunkSumParts;
    static_assert(CH4 % kChunkSumParts == 0, "chunk must split evenly");
    const int tile = blockIdx.x / kChunkSumParts, share = blockIdx.x % kChunkSumParts;
    int4* __restrict__ base = reinterpret_cast<int4*>(chunk_acc) + (size_t)tile * nsplit * CH4;
    for (int e = share * PER + threadIdx.x; e < (share + 1) * PER; e += 256) {
        int4 s = base[e];
        for (int ch = 1; ch < nsplit; ++ch) {
            const int4 v = base[(size_t)ch * CH4 + e];
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
        base[e] = s;
    }
}

// Grouped: every upper-triangular tile of every system in the group; a fixed
// grid loops over them (so the launch can be captured once and replayed).
template <int S, int NL>
__global__ __launch_bounds__(512) void k_gemm_int8x_grouped(const GroupDesc* __restrict__ g) {
    extern __shared__ __align__(16) int8_t smem_raw[];
    I8Smem<S>& sm = *reinterpret_cast<I8Smem<S>*>(smem_raw);
    const int total = g->total_tiles;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int s = group_find(g->tile_off, g->nsys, item);
        const SysView& v = g->sys[s];
        if (v.st->done || v.st->phase != 1) continue;
        int bi = 0, bj = 0, tl = item - g->tile_off[s], nt = v.ld / QB, off = 0;
        while (tl >= off + (nt - bi)) { off += nt - bi; ++bi; }
        bj = bi + (tl - off);
        int8x_tile<S, NL, false, false>(v.buf0, v.buf1, v.ld, v.st, v.digits, v.scale, v.part, bi, bj, sm, nullptr,
                                     nullptr);
        __syncthreads();
    }
}

// Compute units of the current device (cached per device; callers may be on
// several threads).
int device_cus() {
    static std::atomic<int> cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cached[dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

template <int S, int NL, bool THR, bool UPPER, int C = 0>
static hipError_t launch_tile_kernel(SplitScratch& s, double* buf0, double* buf1, int ld, State* st, double* part,
                                     hipStream_t stream, const int* env, int when_full = 0) {
    const int nt = ld / QB;
    const int T = nt * (nt + 1) / 2;
    const size_t lds = sizeof(I8Smem<S, C>);
    static std::atomic<unsigned long long> attr_done{0};
    hipError_t e = once_per_device(attr_done, [&] {
        hipError_t r = hipFuncSetAttribute((const void*)k_gemm_int8x<S, NL, THR, UPPER, C>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (r == hipSuccess && !THR)
            r = hipFuncSetAttribute((const void*)k_gemm_int8x_tail<S, NL, UPPER, C>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        return r;
    });
    if (e != hipSuccess) return e;
    // Tiles of a last wave that would leave at least half of the CUs idle
    // are split along K into nsplit <= 8 chunks (wave quantisation of the
    // tail), when a tile's K loop covers at least 4096 columns: shorter tiles
    // cost less than summing their chunks.
    int t_full = T, nsplit = 1;
    if (!THR && s.tail_split != 0 && s.tail_acc && ld / QK >= 128) {
        const int cus = device_cus();
        const int r = T % cus;
        if (r > 0 && 2 * r <= cus) {
            nsplit = std::min(8, cus / r);
            if (nsplit >= 2 && (size_t)r * nsplit * NL * 2 * 16 * 512 * sizeof(int) <= s.tail_bytes) t_full = T - r;
            else nsplit = 1;
        }
    }
    const int grid = t_full + (T - t_full) * nsplit;
    hipLaunchKernelGGL((k_gemm_int8x<S, NL, THR, UPPER, C>), dim3(grid), dim3(512), lds, stream, buf0, buf1, ld, st,
                       s.digits, s.scale, part, env, s.rmax, s.tile_group, t_full, nsplit, s.tail_acc, when_full);
    if (t_full < T) {
        hipLaunchKernelGGL(k_chunk_sum<NL>, dim3((T - t_full) * kChunkSumParts), dim3(256), 0, stream, s.tail_acc,
                           nsplit, st, when_full);
        hipLaunchKernelGGL((k_gemm_int8x_tail<S, NL, UPPER, C>), dim3(T - t_full), dim3(512), lds, stream, buf0, buf1, ld,
                           st, s.digits, s.scale, part, s.rmax, s.tile_group, t_full, nsplit, s.tail_acc, when_full);
    }
    return hipGetLastError();
}

template <int S, int NL>
static hipError_t launch_list_kernel(SplitScratch& s, double* buf0, double* buf1, int ld, State* st, double* part,
                                     hipStream_t stream, const int* env) {
    const int nt = ld / QB;
    const int T = nt * (nt + 1) / 2;
    const size_t lds = sizeof(I8Smem<S>);
    static std::atomic<unsigned long long> attr_done{0};
    hipError_t e = once_per_device(attr_done, [&] {
        return hipFuncSetAttribute((const void*)k_gemm_int8x_list<S, NL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds);
    });
    if (e != hipSuccess) return e;
    int* list = s.tz + (size_t)2 * T;
    int* ctr = list + T;
    hipLaunchKernelGGL(k_list_reset, dim3(1), dim3(64), 0, stream, ctr, st);
    hipLaunchKernelGGL(k_tile_list, dim3((T + 255) / 256), dim3(256), 0, stream, st, env, s.tz, nt, s.tile_group, part,
                       list, ctr);
    const int grid = std::min(T, device_cus());
    hipLaunchKernelGGL((k_gemm_int8x_list<S, NL>), dim3(grid), dim3(512), lds, stream, buf0, buf1, ld, st, s.digits, s.scale,
                       part, env, s.tz, list, ctr);
    return hipGetLastError();
}

template <int S, int NL>
static hipError_t run_int8x(SplitScratch& s, double* buf0, double* buf1, int ld, State* st, double* part,
                            hipStream_t stream, const int* env) {
    if (env && s.tz) {
        // thresholded: the work-list product, and with the dense switch the
        // dense tile kernel over every upper tile (rows encoded whole); of
        // the two, the first runs while State::full_fill is clear, the second
        // while it is set.  The same tiles get the same integer sums either way.
        hipError_t e = launch_list_kernel<S, NL>(s, buf0, buf1, ld, st, part, stream, env);
        if (e == hipSuccess && s.dense_switch)
            e = launch_tile_kernel<S, NL, false, false>(s, buf0, buf1, ld, st, part, stream, nullptr, 1);
        return e;
    }
    if (env) return launch_tile_kernel<S, NL, true, false>(s, buf0, buf1, ld, st, part, stream, env);
    // dense products: the stage configuration chosen by the autotuner
    if constexpr (i8_cfg_ok(S, 2)) {
        if (s.stage_cfg == 2)
            return s.upper ? launch_tile_kernel<S, NL, false, true, 2>(s, buf0, buf1, ld, st, part, stream, nullptr)
                           : launch_tile_kernel<S, NL, false, false, 2>(s, buf0, buf1, ld, st, part, stream, nullptr);
    }
    if (s.stage_cfg == 1)
        return s.upper ? launch_tile_kernel<S, NL, false, true, 1>(s, buf0, buf1, ld, st, part, stream, nullptr)
                       : launch_tile_kernel<S, NL, false, false, 1>(s, buf0, buf1, ld, st, part, stream, nullptr);
    if (s.upper) return launch_tile_kernel<S, NL, false, true>(s, buf0, buf1, ld, st, part, stream, nullptr);
    return launch_tile_kernel<S, NL, false, false>(s, buf0, buf1, ld, st, part, stream, nullptr);
}

// Thresholded X: one wave per padded row, over the columns of its row panel's
// range of nonzero 32-column blocks only, rounded out to whole K stages the
// way the product rounds its K range (X is zero outside the range, and no
// product reads digits outside it).  Same digits as encode_row.  A panel with
// no nonzero block is read by no product.
template <int S>
__global__ __launch_bounds__(256) void k_encode_int8_env(const double* __restrict__ buf0,
                                                         const double* __restrict__ buf1, int ld,
                                                         const State* __restrict__ st,
                                                         int8_t* __restrict__ digits,
                                                         double* __restrict__ scale, const int* __restrict__ env) {
    if (st->done || st->phase != 1) return;
    constexpr int KS = I8Stage<S>::KS;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (st->full_fill) {   // the dense tile kernel reads every K block
        encode_row<S>(st->cur ? buf1 : buf0, ld, i, lane, digits, scale, 0, ld);
        return;
    }
    const int p = i / QB;
    const int lo = env[2 * p], hi = env[2 * p + 1];
    if (lo > hi) {
        if (lane == 0) scale[i] = 1.0;
        return;
    }
    const int c0 = (lo / KS) * KS * 32, c1 = min(ld, (hi / KS + 1) * KS * 32);
    encode_row<S>(st->cur ? buf1 : buf0, ld, i, lane, digits, scale, c0, c1);
}

template <int S>
static hipError_t run_encode(SplitScratch& s, const double* buf0, const double* buf1, int ld, State* st,
                             hipStream_t stream) {
    if (s.env) {
        hipLaunchKernelGGL(k_encode_int8_env<S>, dim3(ld / 4), dim3(256), 0, stream, buf0, buf1, ld, st, s.digits,
                           s.scale, s.env);
        return hipGetLastError();
    }
    if (s.upper) {
        const int nb = ld / 32;
        hipLaunchKernelGGL(k_encode_int8_upper<S>, dim3(nb * (nb + 1) / 2), dim3(256), 0, stream, buf0, buf1, ld,
                           st, s.digits, s.scale, s.rmax);
    } else if (ld <= 2048 * ENC_CH)
        hipLaunchKernelGGL(k_encode_int8_reg<S>, dim3(ld), dim3(256), 0, stream, buf0, buf1, ld, st, s.digits,
                           s.scale);
    else
        hipLaunchKernelGGL(k_encode_int8<S>, dim3(ld / 4), dim3(256), 0, stream, buf0, buf1, ld, st, s.digits,
                           s.scale);
    return hipGetLastError();
}

template <int S, int NL>
static hipError_t run_grouped(const GroupDesc* g, int gemm_blocks, hipStream_t stream) {
    const size_t lds = sizeof(I8Smem<S>);
    static std::atomic<unsigned long long> attr_done{0};
    hipError_t e = once_per_device(attr_done, [&] {
        return hipFuncSetAttribute((const void*)k_gemm_int8x_grouped<S, NL>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_encode_int8_grouped<S>, dim3(1024), dim3(256), 0, stream, g);
    hipLaunchKernelGGL((k_gemm_int8x_grouped<S, NL>), dim3(gemm_blocks), dim3(512), lds, stream, g);
    return hipGetLastError();
}

hipError_t launch_int8x_grouped(int slices, int levels, const GroupDesc* g, int gemm_blocks, hipStream_t stream) {
    const bool next = levels == slices + 1;
    if (!next && levels != slices) return hipErrorInvalidValue;
    switch (slices) {
        case 2: return next ? run_grouped<2, 3>(g, gemm_blocks, stream) : run_grouped<2, 2>(g, gemm_blocks, stream);
        case 3: return next ? run_grouped<3, 4>(g, gemm_blocks, stream) : run_grouped<3, 3>(g, gemm_blocks, stream);
        case 4: return next ? run_grouped<4, 5>(g, gemm_blocks, stream) : run_grouped<4, 4>(g, gemm_blocks, stream);
        case 5: return next ? run_grouped<5, 6>(g, gemm_blocks, stream) : run_grouped<5, 5>(g, gemm_blocks, stream);
        case 6: return next ? hipErrorInvalidValue : run_grouped<6, 6>(g, gemm_blocks, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_int8x_encode(SplitScratch& s, const double* buf0, const double* buf1, int ld, State* st,
                               hipStream_t stream) {
    switch (s.slices) {
        case 2: return run_encode<2>(s, buf0, buf1, ld, st, stream);
        case 3: return run_encode<3>(s, buf0, buf1, ld, st, stream);
        case 4: return run_encode<4>(s, buf0, buf1, ld, st, stream);
        case 5: return run_encode<5>(s, buf0, buf1, ld, st, stream);
        case 6: return run_encode<6>(s, buf0, buf1, ld, st, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_int8x_gemm(SplitScratch& s, double* buf0, double* buf1, int ld, State* st, double* part,
                             int* nslots, hipStream_t stream, const int* env) {
    const int nt = ld / QB;
    *nslots = nt * (nt + 1) / 2;
    const bool next = s.levels == s.slices + 1;
    if (!next && s.levels != s.slices) return hipErrorInvalidValue;
    switch (s.slices) {
        case 2: return next ? run_int8x<2, 3>(s, buf0, buf1, ld, st, part, stream, env)
                            : run_int8x<2, 2>(s, buf0, buf1, ld, st, part, stream, env);
        case 3: return next ? run_int8x<3, 4>(s, buf0, buf1, ld, st, part, stream, env)
                            : run_int8x<3, 3>(s, buf0, buf1, ld, st, part, stream, env);
        case 4: return next ? run_int8x<4, 5>(s, buf0, buf1, ld, st, part, stream, env)
                            : run_int8x<4, 4>(s, buf0, buf1, ld, st, part, stream, env);
        case 5: return next ? run_int8x<5, 6>(s, buf0, buf1, ld, st, part, stream, env)
                            : run_int8x<5, 5>(s, buf0, buf1, ld, st, part, stream, env);
        case 6: return next ? hipErrorInvalidValue : run_int8x<6, 6>(s, buf0, buf1, ld, st, part, stream, env);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sp2
