// Internal declarations shared by the HIP kernels and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

struct sp2_ctx;
int sp2_ctx_device_of(const sp2_ctx* c);   // defined with the context

namespace sp2 {

constexpr int kMaxIter = 128;      // products per solve (idempotency history)
constexpr int kTile = 128;         // padded leading dimension multiple / GEMM tile

// Device-resident control state of one SP2 solve.  Written only by the
// control kernels (single workgroup), read by every other kernel.
struct State {
    double eps_min, eps_max;
    double t1, t2;              // Tr X_n and Tr X_n^2 (= ||X_n||_F^2) of the current X_n
    double idem[kMaxIter];      // ||X_n^2 - X_n||_F per product
    double fill_min, fill_max;  // block-threshold kept fraction
    float fill[kMaxIter];       // kept fraction after each update (and X_0 at the end slot)
    unsigned long long kept;    // kept-block counter of the current threshold pass
    unsigned long long bits[2]; // branch of each applied update
    int iter;                   // products formed so far
    int branch;                 // branch of the next update (0: X^2, 1: 2X - X^2)
    int done;                   // 0 running, 1 converged, 2 stalled, 3 max_iter,
                                // 4 no resolvable gap at mu, 5 H not finite and symmetric
    int cur;                    // X buffer (0/1) holding X_n
    int result;                 // X buffer holding D once done
    int phase;                  // 0: FP64 products, 1: reduced-precision products, 2: FP32 tail
    int fp64_products;
    int head_switch;
    int tail_left;              // FP32 tail products still to do (BF16X2)
    int full_fill;              // 1 while the kept fraction of X_n is at least
                                // CtrlArgs::dense_fill (thresholded int8 products
                                // then run the dense tile kernel)
};

struct CtrlArgs {
    double n_occ;
    double idem_tol;
    double stall_tol;
    double stall_ratio;   // stall when e_n >= stall_ratio * e_{n-2} (1; 1/2 with a threshold)
    int max_iter;
    int fp64_head;   // products in FP64 before switching phase (-1: never switch)
    int fp32_tail;   // BF16X2: FP32 products after the BF16 stage stalls
    int mixed;       // 0: FP64 only, 1: INT8X, 2: BF16X2, 3: FP32
    double total_blocks;  // block threshold: number of 32 x 32 blocks of N x N (0: off)
    double dense_fill;    // kept fraction from which State::full_fill is set (> 1: never)
};

// ---- grouped (multi-system) launches used by the serving loop ----
constexpr int kMaxGroup = 64;

// One system of a grouped launch: its padded X buffers, int8 digit planes,
// row scales, partial slots, control state and control arguments.
struct SysView {
    double* buf0;
    double* buf1;
    int8_t* digits;
    double* scale;
    double* part;
    State* st;
    int ld;
    int pad_;
    CtrlArgs ctrl;
};

// Work description of a grouped launch (device resident, rewritten by the
// host between ticks).  tile_off / row_off are prefix sums of each system's
// upper-triangular 128 x 128 tiles and of its encode work items (ld / 4).
struct GroupDesc {
    int nsys;
    int total_tiles;
    int total_rowq;
    int pad_;
    int tile_off[kMaxGroup + 1];
    int row_off[kMaxGroup + 1];
    SysView sys[kMaxGroup];
};

#ifdef __HIPCC__
// Index s with off[s] <= item < off[s + 1] (off non-decreasing, n entries + 1).
__device__ __forceinline__ int group_find(const int* off, int n, int item) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
#endif

// Number of upper-triangular tile pairs (bi <= bj) of an nt x nt tile grid.
inline int tri_tiles(int nt) { return nt * (nt + 1) / 2; }

// Canonical slot of tile (bi, bj), bi <= bj: row-major over the upper triangle.
__device__ __forceinline__ int tri_index(int bi, int bj, int nt) {
    return bi * nt - bi * (bi - 1) / 2 + (bj - bi);
}

// Order of the upper-triangular tiles (bi <= bj) of the symmetric product:
// the grid is cut into G x G super-tiles, visited row-major over the upper
// super-triangle, tiles row-major inside each; workgroup ids are dealt so that
// each of the 8 XCDs (which receive workgroups round-robin) owns a contiguous
// run of this order.  Concurrent workgroups of one XCD then share a few row
// panels on both operand sides, which keeps the panels in that XCD's L2.
// Position in the visiting order of workgroup w of a launch of T workgroups:
// each XCD (workgroups are dealt round-robin over the 8 XCDs) gets a
// contiguous run of positions.
__device__ __forceinline__ int xcd_deal(int w, int T) {
    const int q = T >> 3, r = T & 7;
    const int x = w & 7, k = w >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Tile (bi, bj) at position t of the visiting order.  G <= 0: a single
// super-tile (plain row-major order).  G is a launch argument chosen per
// size by sp2_autotune (default 8).
__device__ __forceinline__ void order_tile(int t, int nt, int G, int& bi, int& bj) {
    if (G <= 0 || G > nt) G = nt;
    const int ns = (nt + G - 1) / G;
    for (int I = 0; I < ns; ++I) {
        const int gi = min(G, nt - I * G);
        for (int J = I; J < ns; ++J) {
            const int gj = min(G, nt - J * G);
            const int cnt = (I == J) ? gi * (gi + 1) / 2 : gi * gj;
            if (t < cnt) {
                if (I == J) {
                    int li = 0, off = 0;
                    while (t >= off + (gi - li)) { off += gi - li; ++li; }
                    bi = I * G + li;
                    bj = I * G + li + (t - off);
                } else {
                    bi = I * G + t / gj;
                    bj = J * G + t % gj;
                }
                return;
            }
            t -= cnt;
        }
    }
    bi = bj = 0;   // unreachable for t < nt (nt + 1) / 2
}

__device__ __forceinline__ void tile_of_block(int w, int nt, int G, int& bi, int& bj) {
    order_tile(xcd_deal(w, nt * (nt + 1) / 2), nt, G, bi, bj);
}

// Block mask of a thresholded X, kept after the panel ranges in the env
// buffer (2 nt ints, then nt x mask_words(ld) 64-bit words): for 128-row
// panel p, bit b of words [p W, (p + 1) W) is set when the 32-column block b
// holds a nonzero in some row of the panel.  By symmetry of X it is also the
// set of 32-row blocks with a nonzero in the panel's columns, so a product
// tile (bi, bj) needs exactly the K blocks set in both panels' masks.
__host__ __device__ __forceinline__ int mask_words(int ld) { return (ld / 32 + 63) / 64; }
__host__ __device__ __forceinline__ unsigned long long* env_mask(int* env, int nt) {
    return reinterpret_cast<unsigned long long*>(env + 2 * nt);
}
__host__ __device__ __forceinline__ const unsigned long long* env_mask(const int* env, int nt) {
    return reinterpret_cast<const unsigned long long*>(env + 2 * nt);
}
// Env buffer bytes for nt panels of an ld-wide X.
inline size_t env_bytes(int ld) {
    const int nt = ld / kTile;
    return (size_t)2 * nt * sizeof(int) + (size_t)nt * mask_words(ld) * sizeof(unsigned long long);
}

#ifdef __HIPCC__
// Common block mask of one product tile held in registers: lane l of a wave
// keeps word l of mi & mj (nb / 64 <= 64 words), so finding the next working
// K block in the loop costs a ballot and a lane read, no memory access.
__device__ __forceinline__ unsigned long long common_mask_word(const unsigned long long* __restrict__ mi,
                                                               const unsigned long long* __restrict__ mj, int nb) {
    const int lane = threadIdx.x & 63;
    return lane < ((nb + 63) >> 6) ? (mi[lane] & mj[lane]) : 0ull;
}
// First block >= b (< nb) set in the wave's common mask word mword, or nb.
// Uniform over the wave.
__device__ __forceinline__ int next_block_in_wave(unsigned long long mword, int b, int nb) {
    if (b >= nb) return nb;
    const int lane = threadIdx.x & 63, wd = b >> 6;
    unsigned long long m = lane < wd ? 0ull : mword;
    if (lane == wd) m &= ~0ull << (b & 63);
    const unsigned long long lanes = __ballot(m != 0ull);
    if (lanes == 0ull) return nb;
    const int l = __builtin_ctzll(lanes);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)m, l);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(m >> 32), l);
    const int r = (l << 6) + __builtin_ctzll(((unsigned long long)hi << 32) | lo);
    return r < nb ? r : nb;
}

// The first 32-column block b' >= b (b' < nb) set in both masks mi and mj
// (W words each), or nb.  Uniform in a workgroup.
__device__ __forceinline__ int next_common_block(const unsigned long long* __restrict__ mi,
                                                 const unsigned long long* __restrict__ mj, int b, int nb) {
    if (b >= nb) return nb;
    const int W = (nb + 63) >> 6;
    int wd = b >> 6;
    unsigned long long m = (mi[wd] & mj[wd]) & (~0ull << (b & 63));
    for (;;) {
        if (m) {
            const int r = (wd << 6) + __builtin_ctzll(m);
            return r < nb ? r : nb;
        }
        if (++wd >= W) return nb;
        m = mi[wd] & mj[wd];
    }
}
#endif

// Reading of a degenerate Fermi level: an idempotent X_n whose trace is not
// n_occ, or >= kGapMinIter products without convergence and an idempotency
// error still >= kGapIdem, or eps_max == eps_min, ends the solve with done = 4.
constexpr double kGapIdem = 1.0 / 16.0;
constexpr int kGapMinIter = 100;
// H must be finite and symmetric to within kSymTol * max |H_ij|.
constexpr double kSymTol = 1e-12;
constexpr int kCheckGrid = 2048;   // workgroups (and partial pairs) of the H check
constexpr int kDotBlocks = 2048;   // workgroups (and partials) of the trace-of-product kernel

// ---- launchers (sp2_dense.hip) ----
hipError_t launch_gershgorin(const double* H, int N, double* part, int* nslots, hipStream_t s);
// out[2 b] = max |H_ij - H_ji| (+inf if a non-finite entry was seen),
// out[2 b + 1] = max |H_ij| over the 32 x 32 tile pairs of workgroup b.
hipError_t launch_check_h(const double* H, int N, double* out, int* nout, hipStream_t s);
// Resets the state, sets the Gershgorin bounds and flags an invalid H (done = 5)
// or a flat spectrum (done = 4).
hipError_t launch_bounds(const double* part, int nslots, const double* chk, int nchk, State* st, hipStream_t s);
hipError_t launch_init(const double* H, int N, int ld, double* X0, State* st, double* part,
                       int* nslots, hipStream_t s, unsigned long long* rmax0 = nullptr);
hipError_t launch_ctrl_init(const double* part, int nslots, State* st, CtrlArgs a, hipStream_t s);
hipError_t launch_ctrl_step(const double* part, int nslots, State* st, CtrlArgs a, hipStream_t s);
hipError_t launch_ctrl_step_grouped(const GroupDesc* g, hipStream_t s);
// env (may be null): per 128-row panel p, [env[2p], env[2p+1]] is the range
// of 32-column blocks holding nonzeros of a thresholded X.
// FP64 product.  tail_buf (tail_bytes, may be NULL: no split): chunk
// accumulators of the last-wave tiles split along K, kF64Chunk doubles each;
// 2 x CUs chunks at most.
constexpr size_t kF64Chunk = 16 * 4 * 256;
// split_cap: most chunks per split tile (the autotuner chooses 8 or 16).
// small_ok: a product with ld <= kSmallMaxLd and no threshold runs the
// small-product kernel (32 x 32 tiles), whose partial slots are one per
// 32 x 32 tile (only when no product of another kernel shares the solve's
// slots).  Untuned solves use it up to kSmallLd; the autotuner times it
// against the 128 x 128 kernel up to kSmallMaxLd.
constexpr int kSmallLd = 1024;
constexpr int kSmallMaxLd = 2048;
hipError_t launch_gemm_f64(double* buf0, double* buf1, int ld, State* st, double* part,
                           int* nslots, hipStream_t s, const int* env = nullptr, int tile_group = 8,
                           double* tail_buf = nullptr, size_t tail_bytes = 0, int split_cap = 16,
                           bool small_ok = false);
// Kernel attributes (the dynamic LDS limit) are set per device: `done` holds
// one bit per device id below 64 on which `set()` has succeeded (higher ids
// call it every time).
template <typename F>
hipError_t once_per_device(std::atomic<unsigned long long>& done, F set) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return set();
    const unsigned long long bit = 1ull << dev;
    if (done.load(std::memory_order_acquire) & bit) return hipSuccess;
    e = set();
    if (e == hipSuccess) done.fetch_or(bit, std::memory_order_acq_rel);
    return e;
}
// compute units of the current device (cached on first use)
int device_cus();
hipError_t launch_finalize(const double* buf0, const double* buf1, int ld, int N, double* D,
                           const State* st, hipStream_t s);
// D from the upper triangle of the result buffer (upper-only int8 products).
hipError_t launch_finalize_upper(const double* buf0, const double* buf1, int ld, int N, double* D,
                                 const State* st, hipStream_t s);
// Symmetric pseudo-random ld x ld operand in (-1/2, 1/2) (timing only).
hipError_t launch_fill_test_matrix(double* X, int ld, hipStream_t s);
// int8 matrix-core rate probe: 256 threads per workgroup, iters iterations
// of kInt8RateOpsPerIter ops per wave
constexpr double kInt8RateOpsPerIter = 4.0 * 65536.0;
hipError_t launch_int8_rate(int grid, int iters, double* out, hipStream_t stream);
hipError_t launch_mulliken(const double* D, int n_atoms, double z, double* q, hipStream_t s);
hipError_t launch_dot(const double* A, const double* B, size_t n, double* part, int* nslots,
                      double* out, hipStream_t s);

}  // namespace sp2
