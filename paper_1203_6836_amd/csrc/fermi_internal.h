// Internal declarations of the finite-temperature density matrix (recursive
// Fermi-operator expansion): the elementwise steps and reductions around its
// GEMMs.
#pragma once
#include <hip/hip_runtime.h>

namespace sp2 {

constexpr int kFermiBlocks = 1024;
// X = I/2 - (H - mu I) * scale, scale = beta / 2^(n+2).
hipError_t launch_fermi_init(const double* H, int N, double mu, double scale, double* X, hipStream_t s);
// Newton-Schulz inverse of A = X^2 + (I - X)^2 = I/2 + 2 (X - I/2)^2: with
// |x - 1/2| <= delta over the spectrum of X, A's spectrum lies in
// [1/2, 1/2 + 2 delta^2]; the start Y_0 = c I, c = 2 / (1 + 2 delta^2), leaves
// I - A Y_0 with norm rho = 2 delta^2 / (1 + 2 delta^2) <= 1/3, and after j
// updates the error is rho^(2^j).  The first update Y_1 = Y_0 (2 I - A Y_0) is
// formed without a product; the host adds updates until rho^(2^j) <= kFermiInvErr.
constexpr double kFermiInvErr = 5.5e-16;   // 3^(-32): four updates after Y_1 at delta = 1/2
constexpr int kFermiInvUpdates = 4;        // most updates after Y_1
// A = 2 X2 - 2 X + I, Y = c (2 I - c A).
hipError_t launch_fermi_a(const double* X2, const double* X, int N, double c, double* A, double* Y, hipStream_t s);
// part[2 b], part[2 b + 1] = block b's sums of X_ii and X_ij^2 (fixed order).
hipError_t launch_trace_fro(const double* X, int N, double* part, hipStream_t s);
// out[0], out[1] = fixed-order sums of part[2 k], part[2 k + 1], k < n.
hipError_t launch_sum_pairs(const double* part, int n, double* out, hipStream_t s);

// Chebyshev moments of the entropy: Ht = (H - c I) * inv_w, T0 = I.
hipError_t launch_cheb_init(const double* H, int N, double c, double inv_w, double* Ht, double* T0, hipStream_t s);

}  // namespace sp2
