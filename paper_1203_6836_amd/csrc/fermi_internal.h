// Internal declarations of the finite-temperature density matrix (recursive
// Fermi-operator expansion): the elementwise steps and reductions around its
// GEMMs.
#pragma once
#include <hip/hip_runtime.h>

namespace sp2 {

constexpr int kFermiBlocks = 1024;
// X = I/2 - (H - mu I) * scale, scale = beta / 2^(n+2).
hipError_t launch_fermi_init(const double* H, int N, double mu, double scale, double* X, hipStream_t s);
// Newton-Schulz start of A^(-1): Y_0 = (4/3) I, the best multiple of I for a
// spectrum in [1/2, 1] (|1 - 4 a / 3| <= 1/3); the first update
// Y_1 = Y_0 (2 I - A Y_0) is formed here without a product.
constexpr double kFermiY0 = 4.0 / 3.0;
// Updates after Y_1 (two products each): the error I - A Y_j = (I - A Y_0)^(2^j)
// is at most 3^(-32) ~ 5e-16 after j = 5.
constexpr int kFermiInvUpdates = 4;
// A = 2 X2 - 2 X + I (= X^2 + (I - X)^2), Y = Y_0 (2 I - Y_0 A).
hipError_t launch_fermi_a(const double* X2, const double* X, int N, double* A, double* Y, hipStream_t s);
// R <- 2 I - R in place.
hipError_t launch_two_minus(double* R, int N, hipStream_t s);
// part[2 b], part[2 b + 1] = block b's sums of X_ii and X_ij^2 (fixed order).
hipError_t launch_trace_fro(const double* X, int N, double* part, hipStream_t s);
// out[0], out[1] = fixed-order sums of part[2 k], part[2 k + 1], k < n.
hipError_t launch_sum_pairs(const double* part, int n, double* out, hipStream_t s);

}  // namespace sp2
