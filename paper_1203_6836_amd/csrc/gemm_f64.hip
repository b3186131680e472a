// FP64 matrix products of the non-orthogonal transforms, the Newton-Schulz
// steps of the Loewdin factor and of the Fermi-operator inverse, and the
// Chebyshev recursion of the entropy:
//     C = alpha A^T B + beta C_in + gamma I        (N x N, row-major, ld N).
// C_ij = sum_k A_ki B_kj, so both operands are read as contiguous row
// segments (rows k, columns i or j): for a symmetric A this is A B.  With
// sym the caller asserts that A^T B is symmetric (A and B symmetric and
// commuting, or A^T B = M^T M-like congruences): only the tiles bi <= bj are
// formed and the off-diagonal ones are mirrored, which halves the work and
// makes C exactly symmetric.
//
// Tile 128 x 128 on v_mfma_f64_16x16x4f64, 4 waves of 64 x 64, K staged 16
// at a time through an LDS double buffer with register prefetch (the layout
// of the SP2 product kernel).  A launch whose last wave of tiles would leave
// at least half of the workgroup slots idle splits those tiles along K into
// chunks summed in chunk order by a tail kernel (every tile when all of them
// fill at most half of the slots).  N need not be a multiple of 128: with
// EDGE the loads outside N read zeros and the stores outside N are skipped.
#include <algorithm>
#include <cmath>

#include "gemm_internal.h"
#include "sp2_internal.h"

namespace sp2 {

namespace {

constexpr int TB = 128;   // tile
constexpr int TK = 16;    // k per stage

typedef double d4g __attribute__((ext_vector_type(4)));

// Full-grid tile order: G x G super-tiles row-major, tiles row-major inside.
__device__ __forceinline__ void order_tile_full(int t, int nt, int G, int& bi, int& bj) {
    if (G <= 0 || G > nt) G = nt;
    const int ns = (nt + G - 1) / G;
    for (int I = 0; I < ns; ++I) {
        const int gi = min(G, nt - I * G);
        for (int J = 0; J < ns; ++J) {
            const int gj = min(G, nt - J * G);
            if (t < gi * gj) {
                bi = I * G + t / gj;
                bj = J * G + t % gj;
                return;
            }
            t -= gi * gj;
        }
    }
    bi = bj = 0;   // unreachable for t < nt^2
}

template <bool SYM>
__device__ __forceinline__ void tile_at(int pos, int nt, int G, int& bi, int& bj) {
    if (SYM) order_tile(pos, nt, G, bi, bj);
    else order_tile_full(pos, nt, G, bi, bj);
}

// One 128 x 128 output tile (bi, bj); all 256 threads take part.  kmode 0:
// the whole K loop; 1: stages [kc0, kc1) stored to chunk (d4 [16][256]);
// 2: no K loop, the sum of nchunks chunks (in chunk order), then the epilogue.
template <bool SYM, bool EDGE>
__device__ __forceinline__ void tn_tile(const GemmTN& g, int bi, int bj, int kmode, int kc0, int kc1,
                                        double* __restrict__ chunk, int nchunks) {
    const int N = g.N;
    const double* __restrict__ A = g.A;
    const double* __restrict__ B = g.B;
    const int i0 = bi * TB, j0 = bj * TB;
    __shared__ double As[2][TK][TB];
    __shared__ double Bs[2][TK][TB];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wi = w >> 1, wj = w & 1;
    const int lrow = tid >> 6, lcol = 2 * (tid & 63);
    double2 ra[4], rb[4];
    auto load2 = [&](const double* __restrict__ M, int k, int col) -> double2 {
        if (!EDGE) return *reinterpret_cast<const double2*>(M + (size_t)k * N + col);
        double2 v = make_double2(0.0, 0.0);
        if (k < N) {
            const double* row = M + (size_t)k * N;
            if (col < N) v.x = row[col];
            if (col + 1 < N) v.y = row[col + 1];
        }
        return v;
    };
    auto gload = [&](int k0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            ra[s] = load2(A, k0 + lrow + 4 * s, i0 + lcol);
            rb[s] = load2(B, k0 + lrow + 4 * s, j0 + lcol);
        }
    };
    auto sstore = [&](int stg) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            As[stg][lrow + 4 * s][lcol] = ra[s].x;
            As[stg][lrow + 4 * s][lcol + 1] = ra[s].y;
            Bs[stg][lrow + 4 * s][lcol] = rb[s].x;
            Bs[stg][lrow + 4 * s][lcol + 1] = rb[s].y;
        }
    };
    d4g acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4g{0.0, 0.0, 0.0, 0.0};
    int ks = 0, ke = (N + TK - 1) / TK;
    if (kc1 >= 0) {
        ks = kc0;
        ke = kc1;
    }
    if (kmode == 2) ke = ks;
    auto compute = [&](int stg) {
#pragma unroll
        for (int k4 = 0; k4 < TK / 4; ++k4) {
            const int kr = k4 * 4 + (lane >> 4);
            double av[4], bv[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) av[m] = As[stg][kr][wi * 64 + m * 16 + (lane & 15)];
#pragma unroll
            for (int n = 0; n < 4; ++n) bv[n] = Bs[stg][kr][wj * 64 + n * 16 + (lane & 15)];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m], bv[n], acc[m][n], 0, 0, 0);
        }
    };
    if (ks < ke) {
        gload(ks * TK);
        sstore(0);
        __syncthreads();
        for (int kt = ks; kt < ke; ++kt) {
            const int stg = (kt - ks) & 1;
            if (kt + 1 < ke) gload((kt + 1) * TK);
            compute(stg);
            if (kt + 1 < ke) sstore(stg ^ 1);
            __syncthreads();
        }
    }
    if (kmode == 1) {
        d4g* out = reinterpret_cast<d4g*>(chunk);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) out[(m * 4 + n) * 256 + tid] = acc[m][n];
        return;
    }
    if (kmode == 2) {
        for (int ch = 0; ch < nchunks; ++ch) {
            const d4g* in = reinterpret_cast<const d4g*>(chunk + (size_t)ch * kF64Chunk);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) acc[m][n] += in[(m * 4 + n) * 256 + tid];
        }
    }
    // epilogue.  With sym only the upper triangle is formed (in a diagonal
    // tile too) and mirrored, so C is exactly symmetric: iterations such as
    // the Fermi-operator recursion amplify an antisymmetric part by about an
    // order of magnitude per step.  C_in may be C itself: every element is
    // read and written by one thread, and a mirrored (lower) element is
    // never read
    const double* Cin = g.Cin;
    double* C = g.C;
    const bool diag = SYM && bi == bj;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const int gj = j0 + wj * 64 + n * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // v_mfma_f64_16x16x4f64 result: lane l, element r is row (l >> 4) + 4 r, column l & 15
                const int gi = i0 + wi * 64 + m * 16 + (lane >> 4) + 4 * r;
                if ((EDGE && (gi >= N || gj >= N)) || (diag && gi > gj)) continue;
                double v = g.alpha * acc[m][n][r];
                if (Cin) v += g.beta * Cin[(size_t)gi * N + gj];
                if (gi == gj) v += g.gamma;
                C[(size_t)gi * N + gj] = v;
                if (SYM && gi != gj) C[(size_t)gj * N + gi] = v;
            }
        }
    }
}

template <bool SYM, bool EDGE>
__global__ __launch_bounds__(256, 2) void k_gemm_tn(GemmTN g, int tile_group, int t_full, int nsplit,
                                                    double* __restrict__ chunk) {
    const int nt = (g.N + TB - 1) / TB, w = blockIdx.x;
    const int nk = (g.N + TK - 1) / TK;
    int pos, kmode = 0, kc0 = 0, kc1 = -1;
    double* cacc = nullptr;
    if (w < t_full) {
        pos = xcd_deal(w, t_full);
    } else {
        const int j = w - t_full, p = j / nsplit, ch = j - p * nsplit;
        pos = t_full + p;
        kmode = 1;
        kc0 = ch * nk / nsplit;
        kc1 = (ch + 1) * nk / nsplit;
        cacc = chunk + (size_t)j * kF64Chunk;
    }
    int bi, bj;
    tile_at<SYM>(pos, nt, tile_group, bi, bj);
    tn_tile<SYM, EDGE>(g, bi, bj, kmode, kc0, kc1, cacc, 0);
}

template <bool SYM, bool EDGE>
__global__ __launch_bounds__(256, 2) void k_gemm_tn_tail(GemmTN g, int tile_group, int t_full, int nsplit,
                                                         double* __restrict__ chunk) {
    const int nt = (g.N + TB - 1) / TB, p = blockIdx.x;
    int bi, bj;
    tile_at<SYM>(t_full + p, nt, tile_group, bi, bj);
    tn_tile<SYM, EDGE>(g, bi, bj, 2, 0, -1, chunk + (size_t)p * nsplit * kF64Chunk, nsplit);
}

template <bool SYM, bool EDGE>
hipError_t launch_tn(const GemmTN& g, int tile_group, double* chunk, size_t chunk_bytes, hipStream_t s) {
    const int nt = (g.N + TB - 1) / TB;
    const int T = SYM ? nt * (nt + 1) / 2 : nt * nt;
    const int nk = (g.N + TK - 1) / TK;
    // Split as the SP2 product does: the sparse last wave of a large
    // product, or every tile of a product whose tiles fill at most half of
    // the workgroup slots (two per CU), into about sqrt(1.4 nk) <= 16 chunks.
    int t_full = T, nsplit = 1;
    if (chunk) {
        const int slots = 2 * device_cus();
        int r = 0;
        if (nk >= 256) {
            r = T % slots;
            if (r > 0 && 2 * r <= slots) nsplit = std::min(16, slots / r);
        } else if (2 * T <= slots) {
            r = T;
            nsplit = std::min({16, slots / T, nk, (int)std::lround(std::sqrt(1.4 * nk))});
        }
        if (nsplit >= 2 && (size_t)r * nsplit * kF64Chunk * sizeof(double) <= chunk_bytes) t_full = T - r;
        else nsplit = 1;
    }
    const int grid = t_full + (T - t_full) * nsplit;
    hipLaunchKernelGGL((k_gemm_tn<SYM, EDGE>), dim3(grid), dim3(256), 0, s, g, tile_group, t_full, nsplit, chunk);
    if (t_full < T)
        hipLaunchKernelGGL((k_gemm_tn_tail<SYM, EDGE>), dim3(T - t_full), dim3(256), 0, s, g, tile_group, t_full,
                           nsplit, chunk);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_tn(const GemmTN& g, bool sym, int tile_group, double* chunk, size_t chunk_bytes,
                          hipStream_t s) {
    if (g.N < 1 || !g.A || !g.B || !g.C || (g.beta != 0.0 && !g.Cin)) return hipErrorInvalidValue;
    const bool edge = g.N % TB != 0;
    if (sym) return edge ? launch_tn<true, true>(g, tile_group, chunk, chunk_bytes, s)
                         : launch_tn<true, false>(g, tile_group, chunk, chunk_bytes, s);
    return edge ? launch_tn<false, true>(g, tile_group, chunk, chunk_bytes, s)
                : launch_tn<false, false>(g, tile_group, chunk, chunk_bytes, s);
}

}  // namespace sp2
