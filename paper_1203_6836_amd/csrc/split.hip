// Thresholding of X after each projection (the paper's linear-scaling runs
// zero every element below tau; the block form zeroes whole 32 x 32 blocks
// whose Frobenius norm is below tau) and the operand storage of the
// reduced-precision products.
#include <algorithm>

#include "split_internal.h"

namespace sp2 {

__device__ __forceinline__ double wsum64(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void tri_coords_t(int t, int nt, int& bi, int& bj) {
    int i = 0, off = 0;
    while (t >= off + (nt - i)) { off += nt - i; ++i; }
    bi = i;
    bj = i + (t - off);
}

// One upper-triangular 128 x 128 tile t = (bi, bj) of X (buffer index xb;
// same numbering as the dense product's partial slots), all 256 threads of
// the workgroup (the body contains a barrier); each wave owns four of its
// sixteen 32 x 32 blocks.  Block rule (elem == 0): blocks with ||B||_F < tau
// are zeroed (with their mirror).  Elementwise rule (elem != 0): elements
// with |x| < tau are zeroed (with their mirror; X is stored exactly
// symmetric, so both copies take the same decision), and a block counts as
// kept while any element of it survives.  The tile's trace and ||X||_F^2
// partials are rewritten for the thresholded X; the idempotency partial of
// the product is kept (zeroed for X_0).  FROM_H (the first pass of a
// thresholded solve, H N x N): the tile's X_0 = (eps_max I - H) /
// (eps_max - eps_min) is formed here from H instead of read from X (zero
// outside N x N) and every block is written, the mirror of an off-diagonal
// tile from its upper copy: one pass over H instead of forming X_0 and
// thresholding it in two.
template <bool FROM_H>
__device__ void threshold_tile(double* __restrict__ X, int ld, int N, double tau, int elem, State* __restrict__ st,
                               double* __restrict__ part, int init, int* __restrict__ env, int* __restrict__ tz,
                               int xb, int T, int t, int bi, int bj, const double* __restrict__ H) {
    const bool mirror = bi != bj;
    const double emax = FROM_H ? st->eps_max : 0.0;
    const double inv = FROM_H ? 1.0 / (st->eps_max - st->eps_min) : 0.0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nb = (N + 31) / 32;
    double tr = 0.0, fro = 0.0;
    int kept = 0;
    int kbits = 0;   // column sub-blocks s of row sub-block w (this wave) kept
    // surviving 32-column blocks of panel bi (columns c0) and, by symmetry, of panel bj (rows r0)
    int lo_i = 0x7fffffff, hi_i = -1, lo_j = 0x7fffffff, hi_j = -1;
    // transposed copy of each wave's block, for coalesced writes of the
    // mirrored block (row stride 33 spreads the column-wise stores over banks)
    __shared__ double tb[4][32][33];
    // FROM_H: the wave's four blocks of H are loaded first, all in flight at
    // once (the pass streams the whole matrix); otherwise one block at a time
    double vv[FROM_H ? 4 : 1][16];
    if constexpr (FROM_H) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int b = w * 4 + s, br = b >> 2, bc = b & 3;
            const int r0 = bi * 128 + br * 32, c0 = bj * 128 + bc * 32;
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int e = lane + 64 * m, r = e >> 5, c = e & 31;
                const int i = r0 + r, j = c0 + c;
                vv[s][m] = (i < N && j < N) ? ((i == j ? emax : 0.0) - H[(size_t)i * N + j]) * inv : 0.0;
            }
        }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int b = w * 4 + s, br = b >> 2, bc = b & 3;
        const int r0 = bi * 128 + br * 32, c0 = bj * 128 + bc * 32;
        double* v = vv[FROM_H ? s : 0];
        if constexpr (!FROM_H) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int e = lane + 64 * m, r = e >> 5, c = e & 31;
                v[m] = X[(size_t)(r0 + r) * ld + c0 + c];
            }
        }
        double ss = 0.0;
        bool nz = false, changed = false;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            if (elem && v[m] != 0.0 && fabs(v[m]) < tau) {
                v[m] = 0.0;
                changed = true;
            }
            nz = nz || v[m] != 0.0;
            ss += v[m] * v[m];
        }
        ss = wsum64(ss);
        const bool keep = elem ? __any(nz) : ss >= tau * tau;
        if (!keep && !elem) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                changed = changed || v[m] != 0.0;
                v[m] = 0.0;
            }
        }
        // write back only blocks that changed (every block when X_0 is formed
        // here): the block row by row, and its mirror (X is exactly
        // symmetric, so the mirror is the transpose)
        const bool wchanged = FROM_H || __any(changed);
        if (wchanged) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int e = lane + 64 * m, r = e >> 5, c = e & 31;
                X[(size_t)(r0 + r) * ld + c0 + c] = v[m];
            }
        }
        if (mirror) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int e = lane + 64 * m, r = e >> 5, c = e & 31;
                tb[w][c][r] = v[m];
            }
            __syncthreads();
            if (wchanged) {
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const int e = lane + 64 * m, r = e >> 5, c = e & 31;
                    X[(size_t)(c0 + r) * ld + r0 + c] = tb[w][r][c];
                }
            }
            __syncthreads();
        }
        if (keep) {
            kbits |= 1 << s;
            fro += ss;
            if (r0 == c0) {
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const int e = lane + 64 * m, r = e >> 5, c = e & 31;
                    if (r == c) tr += v[m];
                }
            }
            if ((r0 >> 5) < nb && (c0 >> 5) < nb) kept += 1;
            lo_i = min(lo_i, c0 >> 5);
            hi_i = max(hi_i, c0 >> 5);
            lo_j = min(lo_j, r0 >> 5);
            hi_j = max(hi_j, r0 >> 5);
        }
    }
    tr = wsum64(tr);
    __shared__ double s_tr[4], s_fr[4];
    __shared__ int s_k[4], s_env[4][4], s_bits[4];
    if (lane == 0) {
        s_tr[w] = tr;
        s_fr[w] = fro;
        s_k[w] = kept;
        s_bits[w] = kbits;
        s_env[w][0] = lo_i;
        s_env[w][1] = hi_i;
        s_env[w][2] = lo_j;
        s_env[w][3] = hi_j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double wgt = mirror ? 2.0 : 1.0;
        part[3 * t + 0] = (s_tr[0] + s_tr[1]) + (s_tr[2] + s_tr[3]);
        part[3 * t + 1] = wgt * ((s_fr[0] + s_fr[1]) + (s_fr[2] + s_fr[3]));
        if (init) part[3 * t + 2] = 0.0;
        const int k = s_k[0] + s_k[1] + s_k[2] + s_k[3];
        atomicAdd(&st->kept, (unsigned long long)(mirror ? 2 * k : k));
        if (tz) {
            tz[(size_t)xb * T + t] = k == 0 ? 1 : 0;
            if (init) tz[(size_t)T + t] = 0;
        }
        if (env) {
            int e[4] = {s_env[0][0], s_env[0][1], s_env[0][2], s_env[0][3]};
            for (int q = 1; q < 4; ++q) {
                e[0] = min(e[0], s_env[q][0]);
                e[1] = max(e[1], s_env[q][1]);
                e[2] = min(e[2], s_env[q][2]);
                e[3] = max(e[3], s_env[q][3]);
            }
            if (e[1] >= 0) {
                atomicMin(&env[2 * bi], e[0]);
                atomicMax(&env[2 * bi + 1], e[1]);
                atomicMin(&env[2 * bj], e[2]);
                atomicMax(&env[2 * bj + 1], e[3]);
                // block masks: panel bi gains the kept column sub-blocks
                // (blocks 4 bj .. 4 bj + 3), panel bj the kept row sub-blocks
                const int nt = ld / 128, W = mask_words(ld);
                unsigned long long* mk = env_mask(env, nt);
                int ni = 0, nj = 0;
                for (int q = 0; q < 4; ++q) {
                    ni |= s_bits[q];
                    nj |= (s_bits[q] != 0 ? 1 : 0) << q;
                }
                atomicOr(&mk[(size_t)bi * W + ((4 * bj) >> 6)], (unsigned long long)ni << ((4 * bj) & 63));
                if (mirror)
                    atomicOr(&mk[(size_t)bj * W + ((4 * bi) >> 6)], (unsigned long long)nj << ((4 * bi) & 63));
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_block_threshold(double* __restrict__ buf0, double* __restrict__ buf1,
                                                         int ld, int N, double tau, int elem,
                                                         State* __restrict__ st, double* __restrict__ part,
                                                         int init, int* __restrict__ env, int* __restrict__ tz,
                                                         int when_full) {
    if (st->done || (when_full && !st->full_fill)) return;
    const int xb = init ? 0 : (st->cur ? 0 : 1);
    const int nt = ld / 128;
    const int t = blockIdx.x;
    const int T = nt * (nt + 1) / 2;
    // a tile the product wrote as all zero: nothing to threshold or record
    // (after the dense tile kernel, which writes every tile and no flags,
    // every tile is thresholded and its flag rewritten)
    if (tz && !init && !when_full && tz[(size_t)xb * T + t]) {
        if (threadIdx.x == 0) {
            part[3 * t + 0] = 0.0;
            part[3 * t + 1] = 0.0;
        }
        return;
    }
    int bi, bj;
    tri_coords_t(t, nt, bi, bj);
    threshold_tile<false>(xb == 0 ? buf0 : buf1, ld, N, tau, elem, st, part, init, env, tz, xb, T, t, bi, bj,
                          nullptr);
}

// The X_0 pass of a thresholded solve, X_0 formed from H (N x N) on the fly.
__global__ __launch_bounds__(256) void k_block_threshold_x0(const double* __restrict__ H, double* __restrict__ X,
                                                            int ld, int N, double tau, int elem,
                                                            State* __restrict__ st, double* __restrict__ part,
                                                            int* __restrict__ env, int* __restrict__ tz) {
    if (st->done) return;
    const int nt = ld / 128;
    const int t = blockIdx.x;
    const int T = nt * (nt + 1) / 2;
    int bi, bj;
    tri_coords_t(t, nt, bi, bj);
    threshold_tile<true>(X, ld, N, tau, elem, st, part, 1, env, tz, 0, T, t, bi, bj, H);
}

// Thresholded int8 products driven by a work list (entries (zero_store << 30)
// | (bi << 15) | bj, list_ctr[0] of them): only the tiles the product
// computed are visited.  Every other tile is all zero, with zero partials
// and its flag set, by the list kernel or by the product's zero stores.
__global__ __launch_bounds__(256) void k_block_threshold_list(double* __restrict__ buf0, double* __restrict__ buf1,
                                                              int ld, int N, double tau, int elem,
                                                              State* __restrict__ st, double* __restrict__ part,
                                                              int* __restrict__ env, int* __restrict__ tz,
                                                              const int* __restrict__ list,
                                                              const int* __restrict__ list_ctr) {
    if (st->done || st->full_fill) return;
    const int xb = st->cur ? 0 : 1;
    double* X = xb == 0 ? buf0 : buf1;
    const int nt = ld / 128, T = nt * (nt + 1) / 2;
    const int n = list_ctr[0];
    for (int k = blockIdx.x; k < n; k += gridDim.x) {
        const int it = list[k];
        if (it >> 30) continue;
        const int bi = (it >> 15) & 0x7fff, bj = it & 0x7fff;
        threshold_tile<false>(X, ld, N, tau, elem, st, part, 0, env, tz, xb, T, tri_index(bi, bj, nt), bi, bj, nullptr);
        __syncthreads();   // the tile's shared sums are reused by the next entry
    }
}

// Empty ranges and masks for every panel (before a threshold pass records new ones).
__global__ void k_env_reset(int* __restrict__ env, int npanel, int nwords, const State* __restrict__ st) {
    if (st->done) return;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < npanel) {
        env[2 * p] = 0x7fffffff;
        env[2 * p + 1] = -1;
    }
    if (p < npanel * nwords) env_mask(env, npanel)[p] = 0ull;
}

hipError_t launch_block_threshold(double* buf0, double* buf1, int ld, int N, double tau, int elem, State* st,
                                  double* part, int* nslots, int init, hipStream_t stream, int* env, int* tz,
                                  const int* list, bool dense_switch, const double* H) {
    const int nt = ld / 128;
    const int T = nt * (nt + 1) / 2;
    *nslots = T;
    if (env) {
        const int W = mask_words(ld);
        hipLaunchKernelGGL(k_env_reset, dim3((nt * W + 255) / 256), dim3(256), 0, stream, env, nt, W, st);
    }
    if (list && tz && env && !init) {
        hipLaunchKernelGGL(k_block_threshold_list, dim3(std::min(T, 2048)), dim3(256), 0, stream, buf0, buf1, ld, N,
                           tau, elem, st, part, env, tz, list, list + T);
        if (dense_switch)
            hipLaunchKernelGGL(k_block_threshold, dim3(T), dim3(256), 0, stream, buf0, buf1, ld, N, tau, elem, st,
                               part, 0, env, tz, 1);
    } else {
        if (init && H)
            hipLaunchKernelGGL(k_block_threshold_x0, dim3(T), dim3(256), 0, stream, H, buf0, ld, N, tau, elem, st,
                               part, env, tz);
        else
            hipLaunchKernelGGL(k_block_threshold, dim3(T), dim3(256), 0, stream, buf0, buf1, ld, N, tau, elem, st,
                               part, init, env, tz, 0);
    }
    return hipGetLastError();
}

int split_reserve(SplitScratch& s, int ld, int slices, bool bf16) {
    size_t need = 0;
    need += (size_t)slices * ld * ld;                 // int8 digits
    need += (size_t)ld * sizeof(double) + 256;        // row scales
    need += (size_t)2 * ld * sizeof(unsigned long long) + 256;   // row maxima
    // K-chunk accumulators of split tiles: at most one chunk per CU (256),
    // slices + 1 levels at most
    const size_t tail = slices > 0 ? (size_t)256 * (slices + 1) * 2 * 16 * 512 * sizeof(int) : 0;
    need += tail + 256;
    if (bf16) need += (size_t)2 * ld * ld * sizeof(uint16_t) + (size_t)ld * ld * sizeof(float) + 512;
    if (s.bytes >= need && s.ld == ld && s.slices == slices && s.bf16 == bf16) return 0;
    split_free(s);
    char* base = nullptr;
    if (hipMalloc((void**)&base, need) != hipSuccess) return -2;
    s.bytes = need;
    s.ld = ld;
    s.slices = slices;
    s.bf16 = bf16;
    size_t off = 0;
    s.digits = reinterpret_cast<int8_t*>(base + off);
    off += (size_t)slices * ld * ld;
    off = (off + 255) & ~(size_t)255;
    s.scale = reinterpret_cast<double*>(base + off);
    off += (size_t)ld * sizeof(double);
    off = (off + 255) & ~(size_t)255;
    s.rmax = reinterpret_cast<unsigned long long*>(base + off);
    off += (size_t)2 * ld * sizeof(unsigned long long);
    off = (off + 255) & ~(size_t)255;
    s.tail_acc = tail ? reinterpret_cast<int*>(base + off) : nullptr;
    s.tail_bytes = tail;
    off += tail;
    if (bf16) {
        off = (off + 255) & ~(size_t)255;
        s.bf = reinterpret_cast<uint16_t*>(base + off);
        off += (size_t)2 * ld * ld * sizeof(uint16_t);
        off = (off + 255) & ~(size_t)255;
        s.x32 = reinterpret_cast<float*>(base + off);
    }
    return 0;
}

void split_free(SplitScratch& s) {
    if (s.digits) (void)hipFree(s.digits);
    s = SplitScratch();
}

size_t split_part_slots(int ld) {
    const int nt = ld / 128;
    return (size_t)nt * (nt + 1) / 2;
}

hipError_t launch_split_encode(SplitScratch& s, const double* buf0, const double* buf1, int ld, State* st,
                               hipStream_t stream) {
    if (s.slices > 0) return launch_int8x_encode(s, buf0, buf1, ld, st, stream);
    if (s.bf16) return launch_bf16x2_encode(s, buf0, buf1, ld, st, stream);
    return hipErrorNotSupported;
}
hipError_t launch_split_gemm(SplitScratch& s, double* buf0, double* buf1, int ld, State* st, double* part,
                             int* nslots, hipStream_t stream, const int* env) {
    if (s.slices > 0) return launch_int8x_gemm(s, buf0, buf1, ld, st, part, nslots, stream, env);
    if (s.bf16) return launch_bf16x2_gemm(s, buf0, buf1, ld, st, part, nslots, stream);
    return hipErrorNotSupported;
}

}  // namespace sp2
