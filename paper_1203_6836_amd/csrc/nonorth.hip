// Non-orthogonal formulation (Non-orthogonal formulation subsection): the
// congruence factor Z with Z^T S Z = I (Eq. Congr) is the Loewdin factor
// S^(-1/2), built by the coupled Newton-Schulz iteration
//   Y_0 = S / c, Z_0 = I, T_k = (3 I - Z_k Y_k) / 2, Y_{k+1} = Y_k T_k,
//   Z_{k+1} = T_k Z_k,
// for which Z_k -> (S / c)^(-1/2) quadratically when the spectrum of S / c
// lies in (0, 1] (c = the Gershgorin bound of S).  The products run in the
// FP64 product kernel (symmetric ones for the polynomials in S and the two
// congruences); these kernels do the elementwise steps, the residual
// ||Z_k Y_k - I||_F and the Mulliken charges with the overlap.
#include "nonorth_internal.h"

#include <cmath>

namespace sp2 {

__device__ __forceinline__ double wred_sum_n(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave per row.
__global__ __launch_bounds__(256) void k_row_abs_max(const double* __restrict__ S, int N,
                                                     unsigned long long* __restrict__ mx) {
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= N) return;
    double s = 0.0;
    for (int j = lane; j < N; j += 64) s += fabs(S[(size_t)i * N + j]);
    s = wred_sum_n(s);
    if (lane == 0) atomicMax(mx, (unsigned long long)__double_as_longlong(s));
}

__global__ void k_zero_word(unsigned long long* w) {
    if (threadIdx.x == 0) *w = 0ull;
}

__global__ __launch_bounds__(256) void k_ns_init(const double* __restrict__ S, int N,
                                                 const unsigned long long* __restrict__ mx, double* __restrict__ Y,
                                                 double* __restrict__ Z) {
    const double inv = 1.0 / __longlong_as_double((long long)*mx);
    const size_t n2 = (size_t)N * N;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 256) {
        const size_t i = e / N, j = e % N;
        Y[e] = S[e] * inv;
        Z[e] = i == j ? 1.0 : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_ns_step(double* __restrict__ T, int N, double* __restrict__ part) {
    const size_t n2 = (size_t)N * N;
    double r = 0.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 256) {
        const size_t i = e / N, j = e % N;
        const double t = T[e];
        const double d = t - (i == j ? 1.0 : 0.0);
        r += d * d;
        T[e] = (i == j ? 1.5 : 0.0) - 0.5 * t;
    }
    r = wred_sum_n(r);
    __shared__ double sw[4];
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}

__global__ __launch_bounds__(256) void k_sum_sqrt(const double* __restrict__ part, int n, double* __restrict__ out) {
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) s += part[k];
    s = wred_sum_n(s);
    __shared__ double sw[4];
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = sqrt((sw[0] + sw[1]) + (sw[2] + sw[3]));
}

__global__ __launch_bounds__(256) void k_scale_inv_sqrt(double* __restrict__ Z, int N,
                                                        const unsigned long long* __restrict__ mx) {
    const double f = 1.0 / sqrt(__longlong_as_double((long long)*mx));
    const size_t n2 = (size_t)N * N;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 256) Z[e] *= f;
}

__global__ __launch_bounds__(256) void k_mulliken_overlap(const double* __restrict__ D,
                                                          const double* __restrict__ S, int n_atoms, double z_val,
                                                          double* __restrict__ q) {
    const int a = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (a >= n_atoms) return;
    const int N = 4 * n_atoms;
    double pop = 0.0;
    for (int k = 0; k < 4; ++k) {
        const size_t row = (size_t)(4 * a + k) * N;
        double s = 0.0;
        for (int j = lane; j < N; j += 64) s += D[row + j] * S[row + j];
        pop += wred_sum_n(s);
    }
    if (lane == 0) q[a] = 2.0 * pop - z_val;
}

static int grid_for(size_t n2) {
    const size_t g = (n2 + 255) / 256;
    return (int)(g < 4096 ? g : 4096);
}

hipError_t launch_row_abs_max(const double* S, int N, unsigned long long* mx, hipStream_t s) {
    hipLaunchKernelGGL(k_row_abs_max, dim3((N + 3) / 4), dim3(256), 0, s, S, N, mx);
    return hipGetLastError();
}
hipError_t launch_zero_word(unsigned long long* w, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_word, dim3(1), dim3(64), 0, s, w);
    return hipGetLastError();
}
hipError_t launch_ns_init(const double* S, int N, const unsigned long long* mx, double* Y, double* Z, hipStream_t s) {
    hipLaunchKernelGGL(k_ns_init, dim3(grid_for((size_t)N * N)), dim3(256), 0, s, S, N, mx, Y, Z);
    return hipGetLastError();
}
hipError_t launch_ns_step(double* T, int N, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_ns_step, dim3(kNsBlocks), dim3(256), 0, s, T, N, part);
    return hipGetLastError();
}
hipError_t launch_sum_sqrt(const double* part, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}
hipError_t launch_scale_inv_sqrt(double* Z, int N, const unsigned long long* mx, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(grid_for((size_t)N * N)), dim3(256), 0, s, Z, N, mx);
    return hipGetLastError();
}
hipError_t launch_mulliken_overlap(const double* D, const double* S, int n_atoms, double z_val, double* q,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_mulliken_overlap, dim3((n_atoms + 3) / 4), dim3(256), 0, s, D, S, n_atoms, z_val, q);
    return hipGetLastError();
}

}  // namespace sp2
