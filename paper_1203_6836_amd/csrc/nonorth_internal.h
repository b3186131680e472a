// Internal declarations of the non-orthogonal formulation: the elementwise
// steps of the Loewdin factor's coupled Newton-Schulz iteration and Mulliken
// charges with the overlap.
#pragma once
#include <hip/hip_runtime.h>

namespace sp2 {

// mx[0] <- bit pattern of max_i sum_j |S_ij| (the Gershgorin bound of the
// largest eigenvalue of S); mx[0] must be zeroed first (k order-free: the
// maximum of non-negative doubles compared as bit patterns is exact).
hipError_t launch_row_abs_max(const double* S, int N, unsigned long long* mx, hipStream_t s);
// Zero one 64-bit word (graph-safe, no memset).
hipError_t launch_zero_word(unsigned long long* w, hipStream_t s);
// Y <- S / c with c = the bound in mx, Z <- I (N x N row-major).
hipError_t launch_ns_init(const double* S, int N, const unsigned long long* mx, double* Y, double* Z, hipStream_t s);
// T <- 1.5 I - 0.5 T in place, and part[b] = sum over block b of (T - I)^2
// (fixed grid of kNsBlocks workgroups, fixed order inside each).
constexpr int kNsBlocks = 1024;
hipError_t launch_ns_step(double* T, int N, double* part, hipStream_t s);
// out[0] <- sqrt(sum of part[0 .. n)) in fixed order (one workgroup).
hipError_t launch_sum_sqrt(const double* part, int n, double* out, hipStream_t s);
// Z <- Z / sqrt(c) with c the bound in mx.
hipError_t launch_scale_inv_sqrt(double* Z, int N, const unsigned long long* mx, hipStream_t s);
// q_i = 2 sum_{alpha in i} sum_beta D_{alpha beta} S_{alpha beta} - z_val (S
// symmetric, so the inner sum is (D S)_{alpha alpha}); one wave per atom,
// fixed order.
hipError_t launch_mulliken_overlap(const double* D, const double* S, int n_atoms, double z_val, double* q,
                                   hipStream_t s);

}  // namespace sp2
