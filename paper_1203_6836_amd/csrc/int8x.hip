// Reduced-precision SP2 product on int8 MFMA with exact integer accumulation.
//
// The FP64 master X_n is split row by row into fixed-point digit planes:
// with s_i = 2^e_i >= max_j |X_ij| (a power of two, so the scaling is exact),
// y = X_ij / s_i in (-1, 1) is written as y ~ sum_t d_t 2^-(6 + 7 t) with
// integer digits |d_t| <= 64 taken by successive round-to-nearest of the
// remainder (each remainder is exact in FP64).  Because X is symmetric,
//     (X^2)_ij = sum_k X_ik X_jk ~ s_i s_j sum_{t,u} 2^-(12 + 7(t+u)) sum_k d_t[i,k] d_u[j,k],
// i.e. every digit product reads contiguous rows of the digit planes for both
// operands.  Products with t + u < slices are kept; those of one level L = t+u
// share an int32 accumulator, which is exact (|d| <= 64, at most 6 products
// per level, K <= 65536: |acc| < 2^31).  Levels are combined in FP64 in the
// epilogue, which then applies the SP2 update exactly like the FP64 product.
//
// Work layout, storage and staging: see the comments at the kernels.
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
// One wave per padded row: row scale and `slices` digit planes.
template <int S>
__device__ __forceinline__ void encode_row(const double* __restrict__ X, int ld, int i, int lane, int8_t* __restrict__ digits,
                           double* __restrict__ scale) {
    const double* row = X + (size_t)i * ld;
    double m = 0.0;
    for (int j = 8 * lane; j < ld; j += 512) {
        const double4 a = *reinterpret_cast<const double4*>(row + j);
        const double4 b = *reinterpret_cast<const double4*>(row + j + 4);
        m = fmax(m, fmax(fmax(fabs(a.x), fabs(a.y)), fmax(fabs(a.z), fabs(a.w))));
        m = fmax(m, fmax(fmax(fabs(b.x), fabs(b.y)), fmax(fabs(b.z), fabs(b.w))));
    }
    m = wred_max(m);
    int e = 0;
    if (m > 0.0) (void)frexp(m, &e);     // m = f 2^e, f in [0.5, 1): |X_ij| / 2^e < 1
    const double inv = ldexp(1.0, -e);
    if (lane == 0) scale[i] = ldexp(1.0, e);
    const size_t plane = (size_t)ld * ld;
    const size_t rowblk = (size_t)(i >> 5) * (ld >> 5);
    const int r32 = i & 31;
    for (int j = 8 * lane; j < ld; j += 512) {
        double y[8];
        const double4 a = *reinterpret_cast<const double4*>(row + j);
        const double4 b = *reinterpret_cast<const double4*>(row + j + 4);
        y[0] = a.x * inv; y[1] = a.y * inv; y[2] = a.z * inv; y[3] = a.w * inv;
        y[4] = b.x * inv; y[5] = b.y * inv; y[6] = b.z * inv; y[7] = b.w * inv;
        const size_t off = (rowblk + (j >> 5)) * 1024 + r32 * 32 + 16 * (((j >> 4) & 1) ^ dswz(r32)) + (j & 15);
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const double w = ldexp(1.0, 6 + 7 * t);      // digit weight 2^-(6+7t)
            const double iw = ldexp(1.0, -(6 + 7 * t));
            unsigned long long packed = 0ull;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double d = rint(y[q] * w);        // |d| <= 64
                y[q] -= d * iw;                          // exact remainder
                packed |= (unsigned long long)(uint8_t)(int8_t)d << (8 * q);
            }
            *reinterpret_cast<unsigned long long*>(digits + t * plane + off) = packed;
        }
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
    encode_row<S>(st->cur ? buf1 : buf0, ld, blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63, digits, scale);
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
    int e = 0;
    if (m > 0.0) (void)frexp(m, &e);
    const double inv = ldexp(1.0, -e);
    if (tid == 0) scale[i] = ldexp(1.0, e);
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
#pragma unroll
            for (int t = 0; t < S; ++t) {
                const double wt = ldexp(1.0, 6 + 7 * t);
                const double iw = ldexp(1.0, -(6 + 7 * t));
                unsigned long long packed = 0ull;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const double d = rint(y[q] * wt);
                    y[q] -= d * iw;
                    packed |= (unsigned long long)(uint8_t)(int8_t)d << (8 * q);
                }
                *reinterpret_cast<unsigned long long*>(digits + t * plane + off) = packed;
            }
        }
    }
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
        encode_row<S>(st->cur ? v.buf1 : v.buf0, v.ld, i, threadIdx.x & 63, v.digits, v.scale);
    }
}

// ------------------------------------------------------------------ product
// One 512-thread workgroup per upper-triangular 128 x 128 tile; wave w
// covers rows 32 (w >> 1) .. +32 and columns 64 (w & 1) .. +64 as two 32 x 32
// blocks of v_mfma_i32_32x32x32_i8 per level (S x 2 accumulators of 16
// int32).  Each K stage (32 bytes of k) stages 2 operands x S planes x 4 row
// blocks of 1 KiB through LDS in the blocked layout, double buffered, with
// the next stage's loads in flight in registers.
constexpr int QB = 128;          // tile
constexpr int QK = 32;           // k bytes per stage

#ifndef SP2_I8_DMA
#define SP2_I8_DMA 1
#endif
#ifndef SP2_I8_SCHED
#define SP2_I8_SCHED 2           // 0: compiler's own order; n > 0: read lookahead
#endif
#if SP2_I8_DMA
constexpr int I8_NST = 3;         // LDS ring depth (stages), filled by global->LDS loads
#else
constexpr int I8_NST = 2;
#endif

// The staging ring; after the K loop the same LDS holds half of the finished
// tile, transposed, so the mirrored (lower-triangle) copy is written as
// whole rows instead of one 8-byte element per row.  Row stride 129 doubles
// spreads the column-wise LDS stores over the banks.
constexpr int TR_LD = 129;

template <int S>
struct I8Smem {
    union {
        int8_t buf[I8_NST][2 * S * 4][1024];   // [stage][op * S * 4 + slice * 4 + row block][block]
        double tr[64][TR_LD];                  // [tile column (one half)][tile row]
    };
};

// One 128 x 128 output tile (bi, bj) of one system; all 512 threads of the
// workgroup take part (the body contains barriers).
template <int S, bool THR>
__device__ __forceinline__ void int8x_tile(double* __restrict__ buf0, double* __restrict__ buf1, int ld,
                           const State* __restrict__ st, const int8_t* __restrict__ digits,
                           const double* __restrict__ scale, double* __restrict__ part, int bi, int bj,
                           I8Smem<S>& sm, const int* __restrict__ env) {
    const int nt = ld / QB;
    const int t = tri_index(bi, bj, nt);
    const int i0 = bi * QB, j0 = bj * QB;
    const double* __restrict__ Xc = st->cur ? buf1 : buf0;
    double* __restrict__ Xn = st->cur ? buf0 : buf1;
    const size_t plane = (size_t)ld * ld;
    const int nb = ld >> 5;          // blocks per block row

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;

    constexpr int NBLK = 2 * S * 4;             // 1 KiB blocks per stage
    constexpr int PER = NBLK * 64 / 512;        // 16-byte chunks per thread
    static_assert((NBLK * 64) % 512 == 0, "stage must split evenly over 512 threads");
#if !SP2_I8_DMA
    v4i pre[PER];
    auto gload = [&](int kb) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int c = tid + 512 * m;
            const int blk = c >> 6;
            const int op = blk / (S * 4);
            const int rem = blk - op * (S * 4);
            const int sl = rem >> 2, rb = rem & 3;
            const int grb = ((op ? j0 : i0) >> 5) + rb;
            pre[m] = *reinterpret_cast<const v4i*>(digits + sl * plane + ((size_t)grb * nb + kb) * 1024 +
                                                   16 * (c & 63));
        }
    };
    auto sstore = [&](int stg) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int c = tid + 512 * m;
            *reinterpret_cast<v4i*>(&sm.buf[stg][c >> 6][16 * (c & 63)]) = pre[m];
        }
    };
#endif

    v16i acc[S][2];
#pragma unroll
    for (int L = 0; L < S; ++L)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[L][c][r] = 0;

    // fragment address inside a block: row lane % 32, k-half lane / 32
    const int fr = lane & 31;
    const int foff = fr * 32 + 16 * ((lane >> 5) ^ dswz(fr));
    // K range: all of it, or the overlap of the two panels' surviving column
    // blocks of a thresholded X (one 32-byte stage per 32-column block)
    int ks = 0, nk = ld / QK;
    if (THR) {
        const int lo = max(env[2 * bi], env[2 * bj]), hi = min(env[2 * bi + 1], env[2 * bj + 1]);
        ks = lo;
        nk = lo > hi ? lo : hi + 1;
    }
    // Fragment reads are written in order of first use (B plane 0, the A
    // planes, B planes 1 ..), the products in level order, and the scheduler
    // is held to a pattern of one read per two products that keeps every
    // read LA product pairs ahead of its first use, so a stage starts after
    // 3 + LA reads instead of the whole set.
    auto compute = [&](int stg) {
        auto rdA = [&](int sl) { return *reinterpret_cast<const v4i*>(&sm.buf[stg][sl * 4 + wr][foff]); };
        auto rdB = [&](int uu, int c) {
            return *reinterpret_cast<const v4i*>(&sm.buf[stg][S * 4 + uu * 4 + wc * 2 + c][foff]);
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
            for (int tt = 0; tt < S - uu; ++tt)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[tt + uu][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[tt], b[uu][c], acc[tt + uu][c], 0, 0, 0);
#if SP2_I8_SCHED
        constexpr int LA = SP2_I8_SCHED;                 // lookahead in reads
        constexpr int R = 3 * S, P = S * (S + 1) / 2;   // reads, product pairs
        constexpr int MID = R - 3 - LA;
        __builtin_amdgcn_sched_group_barrier(0x100, 3 + LA, 0);
#pragma unroll
        for (int q = 0; q < MID; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 2 * (P - MID), 0);
#endif
    };
#if SP2_I8_DMA
    // Global -> LDS loads without register staging: wave w moves blocks w,
    // w + 8, ... of a stage, one 1 KiB block per instruction (16 bytes per
    // lane).  Stage kt + 2 is issued while stage kt is multiplied; before
    // reading stage kt a wave lets at most the PER loads of stage kt + 1 stay
    // outstanding, and a barrier then makes every wave's blocks visible.
    auto issue = [&](int kb, int stg) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int blk = w + 8 * m;
            const int op = blk / (S * 4);
            const int rem = blk - op * (S * 4);
            const int sl = rem >> 2, rb = rem & 3;
            const int grb = ((op ? j0 : i0) >> 5) + rb;
            const int8_t* g = digits + sl * plane + ((size_t)grb * nb + kb) * 1024 + 16 * lane;
            __builtin_amdgcn_global_load_lds((const void*)g,
                                             (__attribute__((address_space(3))) void*)&sm.buf[stg][blk][0], 16, 0, 0);
        }
    };
    if (ks < nk) issue(ks, 0);
    if (ks + 1 < nk) issue(ks + 1, 1);
    for (int kt = ks; kt < nk; ++kt) {
        // this wave's blocks of stage kt have landed in LDS once at most the
        // PER loads of stage kt + 1 are outstanding; the bare barrier (no
        // fence, which would wait for every outstanding load) then covers the
        // other waves' blocks, and every wave has finished reading the buffer
        // that stage kt + 2 overwrites
        if (kt + 1 < nk) __builtin_amdgcn_s_waitcnt(0x0F70 | PER);   // vmcnt(PER)
        else __builtin_amdgcn_s_waitcnt(0x0F70);                     // vmcnt(0)
        __builtin_amdgcn_s_barrier();
        if (kt + 2 < nk) issue(kt + 2, (kt + 2 - ks) % I8_NST);
        compute((kt - ks) % I8_NST);
    }
    __syncthreads();
#else
    if (ks < nk) gload(ks);
    if (ks < nk) sstore(0);
    __syncthreads();
    for (int kt = ks; kt < nk; ++kt) {
        const int stg = (kt - ks) & 1;
        if (kt + 1 < nk) gload(kt + 1);
        compute(stg);
        if (kt + 1 < nk) sstore(stg ^ 1);
        __syncthreads();
    }
#endif

    // epilogue: combine levels in FP64, apply the SP2 update, partials
    const int br = st->branch;
    const bool mirror = bi != bj;
    double tr = 0.0, fro = 0.0, idm = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int gj = j0 + wc * 64 + c * 32 + (lane & 31);
        const double sj = scale[gj];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            // v_mfma_i32_32x32x32_i8 result: lane l, element r is row 8 (r/4) + 4 (l/32) + r%4, column l%32
            const int gi = i0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            double v = 0.0;
#pragma unroll
            for (int L = S - 1; L >= 0; --L) v += ldexp((double)acc[L][c][r], -(12 + 7 * L));
            const double p = v * scale[gi] * sj;
            const double x = Xc[(size_t)gi * ld + gj];
            const double xn = br ? 2.0 * x - p : p;
            Xn[(size_t)gi * ld + gj] = xn;
            if (mirror) sm.tr[wc * 32 + (lane & 31)][gi - i0] = xn;
            if (gi == gj) tr += xn;
            fro += xn * xn;
            idm += (p - x) * (p - x);
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
    tr = wred_sum(tr);
    fro = wred_sum(fro);
    idm = wred_sum(idm);
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

template <int S, bool THR>
__global__ __launch_bounds__(512) void k_gemm_int8x(double* __restrict__ buf0, double* __restrict__ buf1,
                                                    int ld, const State* __restrict__ st,
                                                    const int8_t* __restrict__ digits,
                                                    const double* __restrict__ scale,
                                                    double* __restrict__ part, const int* __restrict__ env) {
    if (st->done || st->phase != 1) return;
    extern __shared__ __align__(16) int8_t smem_raw[];
    I8Smem<S>& sm = *reinterpret_cast<I8Smem<S>*>(smem_raw);
    int bi, bj;
    tile_of_block(blockIdx.x, ld / QB, bi, bj);
    int8x_tile<S, THR>(buf0, buf1, ld, st, digits, scale, part, bi, bj, sm, env);
}

// Grouped: every upper-triangular tile of every system in the group; a fixed
// grid loops over them (so the launch can be captured once and replayed).
template <int S>
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
        int8x_tile<S, false>(v.buf0, v.buf1, v.ld, v.st, v.digits, v.scale, v.part, bi, bj, sm, nullptr);
        __syncthreads();
    }
}

template <int S, bool THR>
static hipError_t launch_tile_kernel(SplitScratch& s, double* buf0, double* buf1, int ld, State* st, double* part,
                                     hipStream_t stream, const int* env) {
    const int nt = ld / QB;
    const int T = nt * (nt + 1) / 2;
    const size_t lds = sizeof(I8Smem<S>);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_gemm_int8x<S, THR>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_gemm_int8x<S, THR>), dim3(T), dim3(512), lds, stream, buf0, buf1, ld, st, s.digits,
                       s.scale, part, env);
    return hipGetLastError();
}

template <int S>
static hipError_t run_int8x(SplitScratch& s, double* buf0, double* buf1, int ld, State* st, double* part,
                            hipStream_t stream, const int* env) {
    if (env) return launch_tile_kernel<S, true>(s, buf0, buf1, ld, st, part, stream, env);
    return launch_tile_kernel<S, false>(s, buf0, buf1, ld, st, part, stream, nullptr);
}

template <int S>
static hipError_t run_encode(SplitScratch& s, const double* buf0, const double* buf1, int ld, State* st,
                             hipStream_t stream) {
    if (ld <= 2048 * ENC_CH)
        hipLaunchKernelGGL(k_encode_int8_reg<S>, dim3(ld), dim3(256), 0, stream, buf0, buf1, ld, st, s.digits,
                           s.scale);
    else
        hipLaunchKernelGGL(k_encode_int8<S>, dim3(ld / 4), dim3(256), 0, stream, buf0, buf1, ld, st, s.digits,
                           s.scale);
    return hipGetLastError();
}

template <int S>
static hipError_t run_grouped(const GroupDesc* g, int gemm_blocks, hipStream_t stream) {
    const size_t lds = sizeof(I8Smem<S>);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_gemm_int8x_grouped<S>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k_encode_int8_grouped<S>, dim3(1024), dim3(256), 0, stream, g);
    hipLaunchKernelGGL(k_gemm_int8x_grouped<S>, dim3(gemm_blocks), dim3(512), lds, stream, g);
    return hipGetLastError();
}

hipError_t launch_int8x_grouped(int slices, const GroupDesc* g, int gemm_blocks, hipStream_t stream) {
    switch (slices) {
        case 2: return run_grouped<2>(g, gemm_blocks, stream);
        case 3: return run_grouped<3>(g, gemm_blocks, stream);
        case 4: return run_grouped<4>(g, gemm_blocks, stream);
        case 5: return run_grouped<5>(g, gemm_blocks, stream);
        case 6: return run_grouped<6>(g, gemm_blocks, stream);
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
    switch (s.slices) {
        case 2: return run_int8x<2>(s, buf0, buf1, ld, st, part, stream, env);
        case 3: return run_int8x<3>(s, buf0, buf1, ld, st, part, stream, env);
        case 4: return run_int8x<4>(s, buf0, buf1, ld, st, part, stream, env);
        case 5: return run_int8x<5>(s, buf0, buf1, ld, st, part, stream, env);
        case 6: return run_int8x<6>(s, buf0, buf1, ld, st, part, stream, env);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sp2
