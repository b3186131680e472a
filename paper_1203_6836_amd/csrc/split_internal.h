// Internal declarations of the reduced-precision (split) SP2 products and the
// block threshold.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "sp2_internal.h"

namespace sp2 {

constexpr int kMaxSlices = 6;

// Device operands of the split products, owned by the context.
struct SplitScratch {
    int ld = 0;
    int slices = 0;
    int levels = 0;             // int8 digit-product levels t + u < levels: slices or slices + 1 (set per solve)
    bool bf16 = false;
    int8_t* digits = nullptr;   // slices x ld x ld int8 digit planes
    double* scale = nullptr;    // ld row scales (1 + 2^-7) max_j |X_ij| (1 for a zero row)
    uint16_t* bf = nullptr;     // 2 x ld x ld BF16 hi/lo planes
    float* x32 = nullptr;       // ld x ld FP32 master (BF16X2)
    unsigned long long* rmax = nullptr;  // 2 x ld row maxima of |X| (bit patterns), one row per X buffer
    bool upper = false;         // int8 products write upper tiles only (set per solve)
    int tile_group = 8;         // super-tile size of the product tile order (set per solve)
    int stage_cfg = 0;          // int8 K-stage configuration of dense products (0, 1, 2; set per solve)
    int tail_split = -1;        // split the tiles of a partly filled last wave along K (0: never)
    int* tail_acc = nullptr;    // int32 accumulators of the K chunks of split tiles
    size_t tail_bytes = 0;
    size_t bytes = 0;
    // thresholded solves (set per solve, owned by the context): each row
    // panel's range of nonzero 32-column blocks, and per X buffer and
    // upper-triangular 128 x 128 tile a flag "known to be all zero" (int8
    // products from the first product on only; null otherwise), followed by
    // room for the product's work list (T entries) and 2 counters
    const int* env = nullptr;
    int* tz = nullptr;
    // thresholded int8 products: besides the work-list product, launch the
    // dense tile kernel, which runs (and the work-list kernels return at
    // once) while State::full_fill is set
    bool dense_switch = false;
};

int split_reserve(SplitScratch& s, int ld, int slices, bool bf16);
void split_free(SplitScratch& s);
size_t split_part_slots(int ld);

// Encode the current X_n (buffer st->cur) into the split operands when the
// control state says the next product is a reduced-precision one.
hipError_t launch_split_encode(SplitScratch& s, const double* buf0, const double* buf1, int ld, State* st,
                               hipStream_t stream);
// Reduced-precision product with the fused SP2 update (no-op in FP64 phase).
hipError_t launch_split_gemm(SplitScratch& s, double* buf0, double* buf1, int ld, State* st, double* part,
                             int* nslots, hipStream_t stream, const int* env = nullptr);
// Threshold the freshly written X (X_0 when init != 0, else X_{n+1}): zero
// every 32 x 32 block whose Frobenius norm is below tau (elem == 0) or every
// element below tau (elem != 0); rewrite the trace and norm partials of the
// 128 x 128 tiles (keeping the idempotency partial).  With env non-null, also
// records each panel's range of 32-column blocks that still hold a nonzero
// (reset first), for the products' K ranges.  With tz non-null (2 x T flags,
// T upper-triangular tiles, one row per X buffer): tiles the product marked
// as written all zero are skipped, and every other tile's flag is set to
// whether it is all zero after thresholding; the X_0 pass reads no flags,
// sets those of buffer 0 and clears those of buffer 1.  With list non-null
// as well (the int8 product's work list: T entries, then its entry count),
// updates visit only the tiles the product computed; with dense_switch as
// well, a pass over every tile is launched beside it, and of the two the
// list pass runs while State::full_fill is clear, the full pass while it is
// set (the product then ran the dense tile kernel and built no list).  With
// init and H (N x N) non-null, the X_0 pass forms X_0 from H itself (no
// launch_init before it).
hipError_t launch_block_threshold(double* buf0, double* buf1, int ld, int N, double tau, int elem, State* st,
                                  double* part, int* nslots, int init, hipStream_t stream, int* env = nullptr,
                                  int* tz = nullptr, const int* list = nullptr, bool dense_switch = false,
                                  const double* H = nullptr);

// int8 digit-plane product (int8x.hip)
hipError_t launch_int8x_encode(SplitScratch& s, const double* buf0, const double* buf1, int ld, State* st,
                               hipStream_t stream);
hipError_t launch_int8x_gemm(SplitScratch& s, double* buf0, double* buf1, int ld, State* st, double* part,
                             int* nslots, hipStream_t stream, const int* env = nullptr);

// BF16 hi + lo product (bf16x.hip)
hipError_t launch_bf16x2_encode(SplitScratch& s, const double* buf0, const double* buf1, int ld, State* st,
                                hipStream_t stream);
hipError_t launch_bf16x2_gemm(SplitScratch& s, double* buf0, double* buf1, int ld, State* st, double* part,
                              int* nslots, hipStream_t stream);

// Grouped encode + product over every system of g (fixed grids: 1024 encode
// workgroups, gemm_blocks product workgroups), for the serving loop.
hipError_t launch_int8x_grouped(int slices, int levels, const GroupDesc* g, int gemm_blocks, hipStream_t stream);

}  // namespace sp2
