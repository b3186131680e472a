// Dense SP2 kernels for gfx950: spectral bounds, X_0, the FP64-MFMA
// symmetric product with the fused purification update, the single-workgroup
// control step, and small observables (Mulliken charges, traces).
//
// SP2 (second-order spectral projection, Linear scaling section) builds the
// zero-temperature density matrix theta(mu0 I - H) as a sequence of squarings
// X <- X^2 or X <- 2X - X^2 starting from X_0 = (eps_max I - H)/(eps_max - eps_min).
//
// Layout: the library keeps X in two padded ld x ld row-major FP64 buffers
// (ld = N rounded up to 128, zero outside the N x N corner) used ping-pong;
// the zero padding makes every tile of the product full, with no bounds
// checks in the inner loop, and does not change X^2, traces or norms.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "sp2_internal.h"

namespace sp2 {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Deterministic fixed-order block sum of per-thread values (blockDim 256).
__device__ double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- bounds
// One wave per row i: lo_i = H_ii - sum_{j != i} |H_ij|, hi_i = H_ii + same.
// Each 256-thread workgroup covers 4 rows and writes (min lo, max hi).
__global__ __launch_bounds__(256) void k_gershgorin(const double* __restrict__ H, int N,
                                                     double* __restrict__ part) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = blockIdx.x * 4 + w;
    double lo = 1.0e300, hi = -1.0e300;
    if (i < N) {
        const double* row = H + (size_t)i * N;
        double s = 0.0;
        for (int j = lane; j < N; j += 64) s += fabs(row[j]);
        s = wave_sum(s);
        const double d = row[i];
        const double r = s - fabs(d);
        lo = d - r;
        hi = d + r;
    }
    __shared__ double sl[4], sh[4];
    if (lane == 0) { sl[w] = lo; sh[w] = hi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x + 0] = fmin(fmin(sl[0], sl[1]), fmin(sl[2], sl[3]));
        part[2 * blockIdx.x + 1] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    }
}

// H check: every 32 x 32 tile (bi, bj), bi <= bj, of the upper triangle is
// compared with the transpose of tile (bj, bi) through LDS; a fixed grid of
// workgroups strides over the tiles and keeps running maxima.
__global__ __launch_bounds__(256) void k_check_h(const double* __restrict__ H, int N,
                                                 double* __restrict__ out) {
    __shared__ double A[32][33], B[32][33];
    const int nb = (N + 31) / 32;
    const long long T = (long long)nb * (nb + 1) / 2;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    double dmax = 0.0, amax = 0.0;
    bool bad = false;
    for (long long t = blockIdx.x; t < T; t += gridDim.x) {
        // row bi of the upper triangle starts at bi nb - bi (bi - 1) / 2
        int bi = (int)((2.0 * nb + 1.0 - sqrt((2.0 * nb + 1.0) * (2.0 * nb + 1.0) - 8.0 * (double)t)) / 2.0);
        bi = max(0, min(bi, nb - 1));
        while (bi > 0 && (long long)bi * nb - (long long)bi * (bi - 1) / 2 > t) --bi;
        while (bi + 1 < nb && (long long)(bi + 1) * nb - (long long)(bi + 1) * bi / 2 <= t) ++bi;
        const int bj = bi + (int)(t - ((long long)bi * nb - (long long)bi * (bi - 1) / 2));
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = bi * 32 + r, j = bj * 32 + tx;      // tile (bi, bj)
            const int i2 = bj * 32 + r, j2 = bi * 32 + tx;    // tile (bj, bi)
            A[r][tx] = (i < N && j < N) ? H[(size_t)i * N + j] : 0.0;
            B[r][tx] = (i2 < N && j2 < N) ? H[(size_t)i2 * N + j2] : 0.0;
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const double a = A[r][tx], b = B[tx][r];          // H_ij and H_ji
            if (!isfinite(a) || !isfinite(b)) bad = true;
            else {
                dmax = fmax(dmax, fabs(a - b));
                amax = fmax(amax, fabs(a));
            }
        }
    }
    dmax = wave_max(bad ? INFINITY : dmax);
    amax = wave_max(amax);
    __shared__ double sd[4], sa[4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sd[w] = dmax; sa[w] = amax; }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x + 0] = fmax(fmax(sd[0], sd[1]), fmax(sd[2], sd[3]));
        out[2 * blockIdx.x + 1] = fmax(fmax(sa[0], sa[1]), fmax(sa[2], sa[3]));
    }
}

__global__ __launch_bounds__(256) void k_bounds(const double* __restrict__ part, int nslots,
                                                const double* __restrict__ chk, int nchk,
                                                State* __restrict__ st) {
    double lo = 1.0e300, hi = -1.0e300, dmax = 0.0, amax = 0.0;
    for (int k = threadIdx.x; k < nslots; k += 256) {
        lo = fmin(lo, part[2 * k]);
        hi = fmax(hi, part[2 * k + 1]);
    }
    for (int k = threadIdx.x; k < nchk; k += 256) {
        dmax = fmax(dmax, chk[2 * k]);
        amax = fmax(amax, chk[2 * k + 1]);
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    dmax = wave_max(dmax);
    amax = wave_max(amax);
    __shared__ double sl[4], sh[4], sd[4], sa[4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sl[w] = lo; sh[w] = hi; sd[w] = dmax; sa[w] = amax; }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->eps_min = fmin(fmin(sl[0], sl[1]), fmin(sl[2], sl[3]));
        st->eps_max = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
        const double d = fmax(fmax(sd[0], sd[1]), fmax(sd[2], sd[3]));
        const double m = fmax(fmax(sa[0], sa[1]), fmax(sa[2], sa[3]));
        st->t1 = st->t2 = 0.0;
        st->fill_min = 1.0;
        st->fill_max = 0.0;
        st->bits[0] = st->bits[1] = 0ull;
        st->iter = 0;
        st->branch = 0;
        st->done = 0;
        st->cur = 0;
        st->result = 0;
        st->phase = 0;
        st->fp64_products = 0;
        st->head_switch = -1;
        st->tail_left = 0;
        st->full_fill = 0;
        st->kept = 0ull;
        if (!(d <= kSymTol * m)) st->done = 5;                          // also catches NaN / inf
        else if (!(st->eps_max > st->eps_min)) st->done = 4;            // H = c I: no gap anywhere
    }
    for (int k = threadIdx.x; k < kMaxIter; k += 256) {
        st->idem[k] = 0.0;
        st->fill[k] = 0.0f;
    }
}

// ------------------------------------------------------------------ X_0
// One wave per padded row.  Writes X_0 = (eps_max I - H)/(eps_max - eps_min)
// in the N x N corner and zeros elsewhere; per-workgroup partials
// (Tr X_0, ||X_0||_F^2, 0) into part[3 * block]; with rmax non-null also the
// row maxima max_j |X_0 ij| (as bit patterns) for the upper-only int8 path.
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ H, int N, int ld,
                                              double* __restrict__ X, const State* __restrict__ st,
                                              double* __restrict__ part, unsigned long long* __restrict__ rmax) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = blockIdx.x * 4 + w;            // < ld by construction of the grid
    const double emax = st->eps_max;
    const double inv = 1.0 / (st->eps_max - st->eps_min);
    double tr = 0.0, fro = 0.0, mx = 0.0;
    double* xrow = X + (size_t)i * ld;
    if (i < N) {
        const double* hrow = H + (size_t)i * N;
        for (int j = lane; j < ld; j += 64) {
            double x = 0.0;
            if (j < N) {
                x = ((j == i ? emax : 0.0) - hrow[j]) * inv;
                if (j == i) tr += x;
            }
            xrow[j] = x;
            fro += x * x;
            mx = fmax(mx, fabs(x));
        }
    } else {
        for (int j = lane; j < ld; j += 64) xrow[j] = 0.0;
    }
    if (rmax) {
        mx = wave_max(mx);
        if (lane == 0) rmax[i] = (unsigned long long)__double_as_longlong(mx);
    }
    __shared__ double sh[4];
    const double btr = block_sum256(tr, sh);
    const double bfr = block_sum256(fro, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = btr;
        part[3 * blockIdx.x + 1] = bfr;
        part[3 * blockIdx.x + 2] = 0.0;
    }
}

// --------------------------------------------------------------- control
// Fixed-order reduction of nslots x 3 partials (trace, ||X||^2, ||P - X||^2).
__device__ void reduce3(const double* __restrict__ part, int nslots, double out[3]) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = threadIdx.x; k < nslots; k += 256) {
        a += part[3 * k];
        b += part[3 * k + 1];
        c += part[3 * k + 2];
    }
    __shared__ double sh[4];
    out[0] = block_sum256(a, sh);
    out[1] = block_sum256(b, sh);
    out[2] = block_sum256(c, sh);
}

// Branch rule: X^2 if its trace is at least as close to n_occ as that of
// 2X - X^2 (Tr X^2 = t2, Tr(2X - X^2) = 2 t1 - t2).
__device__ __forceinline__ int choose_branch(double t1, double t2, double nocc) {
    return fabs(t2 - nocc) <= fabs(2.0 * t1 - t2 - nocc) ? 0 : 1;
}

__device__ __forceinline__ void set_bit(State* st, int n, int b) {
    if (n < 128 && b) st->bits[n >> 6] |= (1ull << (n & 63));
}
__device__ __forceinline__ void clear_bit(State* st, int n) {
    if (n < 128) st->bits[n >> 6] &= ~(1ull << (n & 63));
}

// Kept-block fraction of the threshold pass that just ran (if any).
__device__ __forceinline__ double take_fill(State* st, const CtrlArgs& a) {
    if (a.total_blocks <= 0.0) return -1.0;
    const double f = (double)st->kept / a.total_blocks;
    st->kept = 0ull;
    st->full_fill = f >= a.dense_fill ? 1 : 0;
    st->fill_min = fmin(st->fill_min, f);
    st->fill_max = fmax(st->fill_max, f);
    return f;
}

__global__ __launch_bounds__(256) void k_ctrl_init(const double* __restrict__ part, int nslots,
                                                   State* __restrict__ st, CtrlArgs a) {
    double r[3];
    reduce3(part, nslots, r);
    if (threadIdx.x == 0) {
        (void)take_fill(st, a);
        st->t1 = r[0];
        st->t2 = r[1];
        const int b = choose_branch(r[0], r[1], a.n_occ);
        st->branch = b;
        set_bit(st, 0, b);
        // phase 0: FP64 products; 1: the reduced-precision (int8 or BF16)
        // products; 2: FP32 products (mixed 3 throughout)
        st->phase = a.mixed == 3 ? 2 : ((a.mixed != 0 && a.fp64_head == 0) ? 1 : 0);
        if (st->phase == 1) st->head_switch = 0;
    }
}

// After product n: the partials hold Tr X_{n+1}, ||X_{n+1}||_F^2 and
// ||X_n^2 - X_n||_F^2.  Stop rules: e_n < idem_tol (converged, D = X_n);
// n >= 4, e_n >= r e_{n-2}, e_n < stall_tol (stalled at the floor of the
// idempotency error, D = X_n; r = 1, or 1/2 with a threshold, whose floor
// keeps creeping down); n + 1 == max_iter (not converged).  Otherwise X_{n+1} becomes
// current and the next branch is chosen from its traces.
__device__ __forceinline__ void ctrl_step_body(const double* __restrict__ part, int nslots, State* __restrict__ st,
                               const CtrlArgs& a) {
    if (st->done) return;
    double r[3];
    reduce3(part, nslots, r);
    if (threadIdx.x != 0) return;
    const int n = st->iter;
    const double e = sqrt(r[2]);
    st->idem[n] = e;
    const double f = take_fill(st, a);
    if (f >= 0.0) st->fill[n] = (float)f;
    st->iter = n + 1;
    if (st->phase == 0) st->fp64_products += 1;   // FP64 products (the whole solve, or the head)
    const bool stall = n >= 4 && e >= a.stall_ratio * st->idem[n - 2] && e < a.stall_tol;
    // BF16X2 runs its own schedule: a stall of the BF16 stage starts a fixed
    // FP32 tail instead of stopping
    // a projector whose trace is not n_occ could not pick the occupied set:
    // the Fermi level is degenerate (done = 4)
    const int gap_or = fabs(st->t1 - a.n_occ) > 0.5 ? 4 : 0;
    if (e < a.idem_tol || (stall && a.mixed != 2)) {
        st->done = gap_or ? gap_or : ((e < a.idem_tol) ? 1 : 2);
        st->result = st->cur;
        clear_bit(st, n);
        return;
    }
    if (n + 1 >= a.max_iter) {
        st->done = (a.max_iter >= kGapMinIter && e >= kGapIdem) ? 4 : 3;
        st->result = 1 - st->cur;
        return;
    }
    if (a.mixed == 2 && st->phase == 2) {
        // tail product: its update X_{n+1} is applied; after fp32_tail of them, stop
        st->tail_left -= 1;
        if (st->tail_left <= 0) {
            st->done = fabs(r[0] - a.n_occ) > 0.5 ? 4 : 2;
            st->result = 1 - st->cur;
            st->t1 = r[0];
            st->t2 = r[1];
            return;
        }
    }
    if (a.mixed == 2 && st->phase == 1 && stall) {
        if (a.fp32_tail <= 0) {
            st->done = gap_or ? gap_or : 2;
            st->result = st->cur;
            clear_bit(st, n);
            return;
        }
        st->phase = 2;
        st->tail_left = a.fp32_tail;
        st->head_switch = n + 1;
    }
    st->cur = 1 - st->cur;
    st->t1 = r[0];
    st->t2 = r[1];
    const int b = choose_branch(r[0], r[1], a.n_occ);
    st->branch = b;
    set_bit(st, n + 1, b);
    if (a.mixed != 0 && st->phase == 0 && n + 1 >= a.fp64_head && a.fp64_head >= 0) {
        st->phase = 1;
        st->head_switch = n + 1;
    }
}

__global__ __launch_bounds__(256) void k_ctrl_step(const double* __restrict__ part, int nslots,
                                                   State* __restrict__ st, CtrlArgs a) {
    ctrl_step_body(part, nslots, st, a);
}

// One workgroup per system of a grouped launch.
__global__ __launch_bounds__(256) void k_ctrl_step_grouped(const GroupDesc* __restrict__ g) {
    const int s = blockIdx.x;
    if (s >= g->nsys) return;
    const SysView& v = g->sys[s];
    ctrl_step_body(v.part, g->tile_off[s + 1] - g->tile_off[s], v.st, v.ctrl);
}

// ------------------------------------------------- FP64 symmetric product
// P = X X for symmetric X: P_ij = sum_k X_ki X_kj, so both MFMA operands are
// read as contiguous row segments of X (rows k, columns i or j), and only
// tiles with bi <= bj are computed; each is written to (bi,bj) and mirrored.
// Tile 128 x 128, 4 waves in a 2 x 2 arrangement, each wave 64 x 64 as 4 x 4
// blocks of v_mfma_f64_16x16x4f64.  K staged through LDS 16 at a time with
// register prefetch of the next stage (double-buffered LDS).
// Fused epilogue: X_{n+1} = P (branch 0) or 2 X_n - P (branch 1), written to
// the other buffer; per-tile partials Tr X_{n+1}, ||X_{n+1}||_F^2,
// ||P - X_n||_F^2 (off-diagonal tiles count twice) into part[3 * tile].
constexpr int GB = 128;   // tile
constexpr int SB = 32;    // tile of the small-product kernel
constexpr int GK = 16;    // k per stage
constexpr int GS = GB;      // LDS row stride (doubles)
constexpr int F64_NST = 2;  // LDS stages (double buffer: 2 stages x 2 operands x 16 KiB)

// Tile id t -> (bi, bj), bi <= bj, row-major over the upper triangle.
__device__ __forceinline__ void tri_coords(int t, int nt, int& bi, int& bj) {
    int i = 0, off = 0;
    while (t >= off + (nt - i)) { off += nt - i; ++i; }
    bi = i;
    bj = i + (t - off);
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tile ids so tiles sharing row panels share an L2.
__device__ __forceinline__ int xcd_remap(int w, int T) {
    const int q = T >> 3, r = T & 7;
    const int x = w & 7, k = w >> 3;
    return x * q + (x < r ? x : r) + k;
}

// One 128 x 128 output tile (bi, bj); all 256 threads take part.  kmode 0:
// the whole tile; kmode 1: only K stages [kc0, kc1), whose accumulators are
// stored to chunk (one chunk of a tile split along K); kmode 2: no K loop,
// the accumulators are the sum of the nchunks chunks at chunk, added in
// chunk order, then the epilogue.  Chunk layout: d4 [16 blocks][256
// threads] (accumulator block m * 4 + n of each thread), 128 KiB.
template <bool THR>
__device__ __forceinline__ void f64_tile(double* __restrict__ buf0, double* __restrict__ buf1, int ld,
                                         const State* __restrict__ st, double* __restrict__ part,
                                         const int* __restrict__ env, int bi, int bj, int kmode, int kc0,
                                         int kc1, double* __restrict__ chunk, int nchunks) {
    const int nt = ld / GB;
    const int t = tri_index(bi, bj, nt);
    const double* __restrict__ Xc = st->cur ? buf1 : buf0;
    double* __restrict__ Xn = st->cur ? buf0 : buf1;
    const int i0 = bi * GB, j0 = bj * GB;

    // LDS double buffer; each operand row of a stage is one contiguous 1 KiB
    // row segment of X
    __shared__ double As[F64_NST][GK][GS];
    __shared__ double Bs[F64_NST][GK][GS];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wi = w >> 1, wj = w & 1;

    // global -> register staging: 4 double2 per operand per thread (loads
    // straight into LDS were measured slower for FP64)
    const int lrow = tid >> 6;           // + 4*s
    const int lcol = 2 * (tid & 63);
    double2 ra[4], rb[4];
    auto gload = [&](int k0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const size_t off = (size_t)(k0 + lrow + 4 * s) * ld;
            ra[s] = *reinterpret_cast<const double2*>(Xc + off + i0 + lcol);
            rb[s] = *reinterpret_cast<const double2*>(Xc + off + j0 + lcol);
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

    d4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    // K stages: all of them (or the chunk [kc0, kc1)), or for a thresholded X
    // the 16-wide stages of the 32-column blocks set in both row panels'
    // block masks (elsewhere one of the two operands is zero, so skipping
    // those stages leaves every sum bitwise unchanged)
    int ks = 0, ke = ld / GK;
    if (kc1 >= 0) {
        ks = kc0;
        ke = kc1;
    }
    if (kmode == 2) ke = ks;                   // accumulators come from the chunks
    const int nbk = ld / 32;
    unsigned long long mword = 0ull;
    if (THR) {
        const unsigned long long* mk = env_mask(env, nt);
        mword = common_mask_word(mk + (size_t)bi * mask_words(ld), mk + (size_t)bj * mask_words(ld), nbk);
    }
    auto next_stage = [&](int s) -> int {      // first working stage >= s, or ke
        if (!THR || s >= ke) return s;
        const int b = next_block_in_wave(mword, s >> 1, nbk);
        return b >= nbk ? ke : max(s, 2 * b);
    };
    auto compute = [&](int stg) {
#pragma unroll
        for (int k4 = 0; k4 < GK / 4; ++k4) {
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
    int kt = next_stage(ks);
    if (kt < ke) {
        gload(kt * GK);
        sstore(0);
        __syncthreads();
        int stg = 0;
        while (kt < ke) {
            const int kn = next_stage(kt + 1);
            if (kn < ke) gload(kn * GK);
            compute(stg);
            if (kn < ke) sstore(stg ^ 1);
            __syncthreads();
            stg ^= 1;
            kt = kn;
        }
    }

    if (kmode == 1) {
        d4* out = reinterpret_cast<d4*>(chunk);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) out[(m * 4 + n) * 256 + tid] = acc[m][n];
        return;
    }
    if (kmode == 2) {
        for (int ch = 0; ch < nchunks; ++ch) {
            const d4* in = reinterpret_cast<const d4*>(chunk + (size_t)ch * kF64Chunk);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) acc[m][n] += in[(m * 4 + n) * 256 + tid];
        }
    }

    // fused SP2 update + partials
    const int br = st->branch;
    const bool mirror = bi != bj;
    double tr = 0.0, fro = 0.0, idm = 0.0;
    // one straight-line body per mirrored flag: it is uniform, and branching
    // on it per element keeps many values live across blocks
    auto epilogue = [&](auto mirc) {
        constexpr bool MIR = decltype(mirc)::value;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const int gj = j0 + wj * 64 + n * 16 + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // v_mfma_f64_16x16x4f64 result: lane l, element r is row (l >> 4) + 4 r, column l & 15
                    const int gi = i0 + wi * 64 + m * 16 + (lane >> 4) + 4 * r;
                    const double p = acc[m][n][r];
                    const double x = Xc[(size_t)gi * ld + gj];
                    const double xn = br ? 2.0 * x - p : p;
                    Xn[(size_t)gi * ld + gj] = xn;
                    if constexpr (MIR) Xn[(size_t)gj * ld + gi] = xn;
                    tr += gi == gj ? xn : 0.0;
                    fro += xn * xn;
                    idm += (p - x) * (p - x);
                }
            }
        }
    };
    if (mirror) epilogue(std::true_type{});
    else epilogue(std::false_type{});
    const double wgt = mirror ? 2.0 : 1.0;
    __shared__ double sh[4];
    const double btr = block_sum256(tr, sh);
    const double bfr = block_sum256(fro, sh);
    const double bid = block_sum256(idm, sh);
    if (tid == 0) {
        part[3 * t + 0] = btr;
        part[3 * t + 1] = wgt * bfr;
        part[3 * t + 2] = wgt * bid;
    }
}

// At most 256 registers per lane: the accumulators then stay in VGPR form
// (with the whole register file the compiler splits them between VGPRs and
// AGPRs and copies them across on every K stage) and two workgroups fit on
// a CU (LDS 64 KiB each), so one hides the other's barriers and epilogue.
// Workgroups [0, t_full): whole tiles at visiting positions [0, t_full),
// dealt over the XCDs.  Workgroups from t_full on: the tiles at positions
// t_full, t_full + 1, ... (the last, partly filled wave of a launch), each
// split into nsplit chunks of the K loop whose accumulators go to chunk;
// k_gemm_f64_tail finishes them.
template <bool THR>
__global__ __launch_bounds__(256, 2) void k_gemm_f64(double* __restrict__ buf0,
                                                     double* __restrict__ buf1, int ld,
                                                     const State* __restrict__ st,
                                                     double* __restrict__ part,
                                                     const int* __restrict__ env, int tile_group, int t_full,
                                                     int nsplit, double* __restrict__ chunk) {
    if (st->done || st->phase != 0) return;
    const int nt = ld / GB, w = blockIdx.x;
    int pos, kmode = 0, kc0 = 0, kc1 = -1;
    double* cacc = nullptr;
    if (w < t_full) {
        pos = xcd_deal(w, t_full);
    } else {
        const int j = w - t_full, p = j / nsplit, ch = j - p * nsplit, nk = ld / GK;
        pos = t_full + p;
        kmode = 1;
        kc0 = ch * nk / nsplit;
        kc1 = (ch + 1) * nk / nsplit;
        cacc = chunk + (size_t)j * kF64Chunk;
    }
    int bi, bj;
    order_tile(pos, nt, tile_group, bi, bj);
    f64_tile<THR>(buf0, buf1, ld, st, part, env, bi, bj, kmode, kc0, kc1, cacc, 0);
}

// Small products (ld <= kSmallMaxLd; at ld <= 1024 X is at most 8 MiB and
// stays in L2): the 128 x 128 tiles would occupy a handful of CUs, each
// walking its K loop alone, and splitting them along K adds a second launch
// that reads the chunks back.  Instead one workgroup per 32 x 32 upper tile (T = nt(nt+1)/2,
// nt = ld / 32): each of its four waves multiplies a quarter of the K range
// with operands loaded straight into registers (lane l of a 4-deep k step
// reads row k + l / 16 of X, 16 consecutive columns per 16 lanes), the four
// partial tiles are added in LDS in wave order, and the fused update and the
// partials follow as in the large kernel (one slot per 32 x 32 tile).
__global__ __launch_bounds__(256) void k_gemm_f64_small(double* __restrict__ buf0, double* __restrict__ buf1,
                                                        int ld, const State* __restrict__ st,
                                                        double* __restrict__ part) {
    if (st->done || st->phase != 0) return;
    const int nts = ld / SB;
    int t = blockIdx.x, bi = 0;
    while (t >= nts - bi) {
        t -= nts - bi;
        ++bi;
    }
    const int bj = bi + t;
    const double* __restrict__ Xc = st->cur ? buf1 : buf0;
    double* __restrict__ Xn = st->cur ? buf0 : buf1;
    const int i0 = bi * SB, j0 = bj * SB;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int ci = lane & 15, kr = lane >> 4;
    const int kq = ld / 4, k0 = w * kq;    // ld is a multiple of 128: kq of 4
    d4 acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k = k0; k < k0 + kq; k += 4) {
        const double* __restrict__ row = Xc + (size_t)(k + kr) * ld;
        const double a0 = row[i0 + ci], a1 = row[i0 + 16 + ci];
        const double b0 = row[j0 + ci], b1 = row[j0 + 16 + ci];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __shared__ double red[4][SB][SB + 1];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r)   // lane l, element r: row l / 16 + 4 r, column l % 16
                red[w][m * 16 + kr + 4 * r][n * 16 + ci] = acc[m][n][r];
    __syncthreads();
    const int br = st->branch;
    const bool mirror = bi != bj;
    double tr = 0.0, fro = 0.0, idm = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = tid + 256 * q, r = e >> 5, c = e & 31;
        const double p = ((red[0][r][c] + red[1][r][c]) + red[2][r][c]) + red[3][r][c];
        const int gi = i0 + r, gj = j0 + c;
        const double x = Xc[(size_t)gi * ld + gj];
        const double xn = br ? 2.0 * x - p : p;
        Xn[(size_t)gi * ld + gj] = xn;
        if (mirror) Xn[(size_t)gj * ld + gi] = xn;
        tr += gi == gj ? xn : 0.0;
        fro += xn * xn;
        idm += (p - x) * (p - x);
    }
    const double wgt = mirror ? 2.0 : 1.0;
    __shared__ double sh[4];
    const double btr = block_sum256(tr, sh);
    const double bfr = block_sum256(fro, sh);
    const double bid = block_sum256(idm, sh);
    if (tid == 0) {
        part[3 * blockIdx.x + 0] = btr;
        part[3 * blockIdx.x + 1] = wgt * bfr;
        part[3 * blockIdx.x + 2] = wgt * bid;
    }
}

// Epilogue of the split tiles: workgroup p sums the nsplit chunks of the tile
// at visiting position t_full + p and applies the update.
__global__ __launch_bounds__(256, 2) void k_gemm_f64_tail(double* __restrict__ buf0, double* __restrict__ buf1,
                                                          int ld, const State* __restrict__ st,
                                                          double* __restrict__ part, int tile_group, int t_full,
                                                          int nsplit, double* __restrict__ chunk) {
    if (st->done || st->phase != 0) return;
    const int nt = ld / GB, p = blockIdx.x;
    int bi, bj;
    order_tile(t_full + p, nt, tile_group, bi, bj);
    f64_tile<false>(buf0, buf1, ld, st, part, nullptr, bi, bj, 2, 0, -1, chunk + (size_t)p * nsplit * kF64Chunk,
                    nsplit);
}

// ---------------------------------------------------------------- finalize
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ buf0,
                                                  const double* __restrict__ buf1, int ld, int N,
                                                  double* __restrict__ D,
                                                  const State* __restrict__ st) {
    const double* X = st->result ? buf1 : buf0;
    const size_t total = (size_t)N * N;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const size_t i = e / N, j = e - i * N;
        D[e] = X[i * ld + j];
    }
}

// D from an X whose upper triangle (32 x 32 blocks I <= J) is valid: each
// workgroup copies block (I, J) and its transpose (through LDS) to D.
__global__ __launch_bounds__(256) void k_finalize_upper(const double* __restrict__ buf0,
                                                        const double* __restrict__ buf1, int ld, int N,
                                                        double* __restrict__ D,
                                                        const State* __restrict__ st) {
    const double* X = st->result ? buf1 : buf0;
    const int nb = (N + 31) / 32;
    const int t = blockIdx.x;
    int I = (int)((2.0 * nb + 1.0 - sqrt((2.0 * nb + 1.0) * (2.0 * nb + 1.0) - 8.0 * (double)t)) / 2.0);
    I = max(0, min(I, nb - 1));
    while (I > 0 && I * nb - I * (I - 1) / 2 > t) --I;
    while (I + 1 < nb && (I + 1) * nb - (I + 1) * I / 2 <= t) ++I;
    const int J = I + (t - (I * nb - I * (I - 1) / 2));
    __shared__ double T[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = I * 32 + r, j = J * 32 + tx;      // i, j < ld: X is padded with zeros
        const double x = X[(size_t)i * ld + j];
        T[r][tx] = x;
        if (i < N && j < N) D[(size_t)i * N + j] = x;
    }
    if (I == J) return;
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = J * 32 + r, j = I * 32 + tx;
        if (i < N && j < N) D[(size_t)i * N + j] = T[tx][r];
    }
}

// Symmetric test operand for timing (the autotuner): X_ij = X_ji in (-1/2, 1/2)
// from an integer hash of (min(i, j), max(i, j)), so that products switch as
// many bits (and draw as much power) as on real data.
__global__ __launch_bounds__(256) void k_fill_test_matrix(double* __restrict__ X, int ld) {
    const size_t total = (size_t)ld * ld;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const unsigned i = (unsigned)(e / ld), j = (unsigned)(e % ld);
        unsigned h = (i < j ? i : j) * 0x9E3779B1u ^ (i < j ? j : i) * 0x85EBCA77u;
        h ^= h >> 15;
        h *= 0x2C1B3C6Du;
        h ^= h >> 12;
        X[e] = (double)(h >> 8) / 16777216.0 - 0.5;
    }
}

// ------------------------------------------------------------ observables
__global__ __launch_bounds__(256) void k_mulliken(const double* __restrict__ D, int n_atoms,
                                                  double z, double* __restrict__ q) {
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= n_atoms) return;
    const size_t N = 4 * (size_t)n_atoms;
    double s = 0.0;
    for (int k = 0; k < 4; ++k) {
        const size_t o = 4 * (size_t)a + k;
        s += D[o * N + o];
    }
    q[a] = 2.0 * s - z;
}

// sum_e A[e] B[e] with a fixed grid of 512 workgroups, then a one-workgroup
// fixed-order reduction into *out (device).
// Partial sums of sum_e A_e B_e, one per workgroup, in a fixed order;
// 16-byte loads when both operands are 16-byte aligned.
template <bool VEC>
__global__ __launch_bounds__(256) void k_dot_part(const double* __restrict__ A,
                                                  const double* __restrict__ B, size_t n,
                                                  double* __restrict__ part) {
    double s = 0.0;
    const size_t stride = (size_t)kDotBlocks * 256;
    if (VEC) {
        const double2* __restrict__ A2 = reinterpret_cast<const double2*>(A);
        const double2* __restrict__ B2 = reinterpret_cast<const double2*>(B);
        for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n / 2; e += stride) {
            const double2 a = A2[e], b = B2[e];
            s += a.x * b.x;
            s += a.y * b.y;
        }
        if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) s += A[n - 1] * B[n - 1];
    } else {
        for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += stride) s += A[e] * B[e];
    }
    __shared__ double sh[4];
    const double b = block_sum256(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}
__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ part, int nslots,
                                                   double* __restrict__ out) {
    double s = 0.0;
    for (int k = threadIdx.x; k < nslots; k += 256) s += part[k];
    __shared__ double sh[4];
    const double b = block_sum256(s, sh);
    if (threadIdx.x == 0) *out = b;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_gershgorin(const double* H, int N, double* part, int* nslots, hipStream_t s) {
    const int g = (N + 3) / 4;
    *nslots = g;
    hipLaunchKernelGGL(k_gershgorin, dim3(g), dim3(256), 0, s, H, N, part);
    return hipGetLastError();
}
hipError_t launch_check_h(const double* H, int N, double* out, int* nout, hipStream_t s) {
    const long long nb = (N + 31) / 32;
    const int g = (int)std::min<long long>(nb * (nb + 1) / 2, kCheckGrid);
    *nout = g;
    hipLaunchKernelGGL(k_check_h, dim3(g), dim3(256), 0, s, H, N, out);
    return hipGetLastError();
}
hipError_t launch_bounds(const double* part, int nslots, const double* chk, int nchk, State* st, hipStream_t s) {
    hipLaunchKernelGGL(k_bounds, dim3(1), dim3(256), 0, s, part, nslots, chk, nchk, st);
    return hipGetLastError();
}
hipError_t launch_init(const double* H, int N, int ld, double* X0, State* st, double* part,
                       int* nslots, hipStream_t s, unsigned long long* rmax0) {
    const int g = ld / 4;
    *nslots = g;
    hipLaunchKernelGGL(k_init, dim3(g), dim3(256), 0, s, H, N, ld, X0, st, part, rmax0);
    return hipGetLastError();
}
hipError_t launch_ctrl_init(const double* part, int nslots, State* st, CtrlArgs a, hipStream_t s) {
    hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(256), 0, s, part, nslots, st, a);
    return hipGetLastError();
}
hipError_t launch_ctrl_step(const double* part, int nslots, State* st, CtrlArgs a, hipStream_t s) {
    hipLaunchKernelGGL(k_ctrl_step, dim3(1), dim3(256), 0, s, part, nslots, st, a);
    return hipGetLastError();
}
hipError_t launch_ctrl_step_grouped(const GroupDesc* g, hipStream_t s) {
    hipLaunchKernelGGL(k_ctrl_step_grouped, dim3(kMaxGroup), dim3(256), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_gemm_f64(double* buf0, double* buf1, int ld, State* st, double* part,
                           int* nslots, hipStream_t s, const int* env, int tile_group, double* tail_buf,
                           size_t tail_bytes, int split_cap, bool small_ok) {
    if (small_ok && !env && ld <= kSmallMaxLd) {
        const int T = tri_tiles(ld / SB);
        *nslots = T;
        hipLaunchKernelGGL(k_gemm_f64_small, dim3(T), dim3(256), 0, s, buf0, buf1, ld, st, part);
        return hipGetLastError();
    }
    const int nt = ld / GB;
    const int T = tri_tiles(nt);
    *nslots = T;
    // Tiles of a last wave that would leave at least half of the workgroup
    // slots (two per CU) idle are split along K into nsplit <= 16 chunks,
    // when a tile's K loop covers at least 4096 columns.  A smaller product
    // whose tiles fill at most half of the slots is latency-bound (each
    // workgroup walks its K stages one after another): all of its tiles are
    // split.  The chunk count balances the stages a chunk walks (~2.8 us
    // each) against the chunks the tail kernel reads back one after another
    // (~2 us each): about sqrt(1.4 nk), at most split_cap and no more than fit.
    int t_full = T, nsplit = 1;
    if (!env && tail_buf) {
        const int slots = 2 * device_cus();
        const int nk = ld / GK;
        int r = 0;
        if (nk >= 256) {
            r = T % slots;
            if (r > 0 && 2 * r <= slots) nsplit = std::min(split_cap, slots / r);
        } else if (2 * T <= slots) {
            r = T;
            nsplit = std::min({split_cap, slots / T, nk, (int)std::lround(std::sqrt(1.4 * nk))});
        }
        if (nsplit >= 2 && (size_t)r * nsplit * kF64Chunk * sizeof(double) <= tail_bytes) t_full = T - r;
        else nsplit = 1;
    }
    const int grid = t_full + (T - t_full) * nsplit;
    if (env)
        hipLaunchKernelGGL(k_gemm_f64<true>, dim3(grid), dim3(256), 0, s, buf0, buf1, ld, st, part, env, tile_group,
                           t_full, nsplit, tail_buf);
    else
        hipLaunchKernelGGL(k_gemm_f64<false>, dim3(grid), dim3(256), 0, s, buf0, buf1, ld, st, part, env,
                           tile_group, t_full, nsplit, tail_buf);
    if (t_full < T)
        hipLaunchKernelGGL(k_gemm_f64_tail, dim3(T - t_full), dim3(256), 0, s, buf0, buf1, ld, st, part, tile_group,
                           t_full, nsplit, tail_buf);
    return hipGetLastError();
}
hipError_t launch_finalize(const double* buf0, const double* buf1, int ld, int N, double* D,
                           const State* st, hipStream_t s) {
    size_t total = (size_t)N * N;
    int g = (int)((total + 255) / 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_finalize, dim3(g), dim3(256), 0, s, buf0, buf1, ld, N, D, st);
    return hipGetLastError();
}
hipError_t launch_finalize_upper(const double* buf0, const double* buf1, int ld, int N, double* D,
                                 const State* st, hipStream_t s) {
    const int nb = (N + 31) / 32;
    hipLaunchKernelGGL(k_finalize_upper, dim3(nb * (nb + 1) / 2), dim3(256), 0, s, buf0, buf1, ld, N, D, st);
    return hipGetLastError();
}
hipError_t launch_fill_test_matrix(double* X, int ld, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_test_matrix, dim3(2048), dim3(256), 0, s, X, ld);
    return hipGetLastError();
}
hipError_t launch_mulliken(const double* D, int n_atoms, double z, double* q, hipStream_t s) {
    hipLaunchKernelGGL(k_mulliken, dim3((n_atoms + 255) / 256), dim3(256), 0, s, D, n_atoms, z, q);
    return hipGetLastError();
}
hipError_t launch_dot(const double* A, const double* B, size_t n, double* part, int* nslots,
                      double* out, hipStream_t s) {
    *nslots = kDotBlocks;
    if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) % 16 == 0)
        hipLaunchKernelGGL(k_dot_part<true>, dim3(kDotBlocks), dim3(256), 0, s, A, B, n, part);
    else
        hipLaunchKernelGGL(k_dot_part<false>, dim3(kDotBlocks), dim3(256), 0, s, A, B, n, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, part, kDotBlocks, out);
    return hipGetLastError();
}

}  // namespace sp2
