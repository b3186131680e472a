// Non-orthogonal formulation (Non-orthogonal formulation subsection): the
// congruence factor Z with Z^T S Z = I (Eq. Congr) is the Loewdin factor
// S^(-1/2), built by the coupled Newton-Schulz iteration
//   Y_0 = S / c, Z_0 = I, T_k = (3 I - Z_k Y_k) / 2, Y_{k+1} = Y_k T_k,
//   Z_{k+1} = T_k Z_k,
// for which Z_k -> (S / c)^(-1/2) quadratically when the spectrum of S / c
// lies in (0, 1] (c = the Gershgorin bound of S).  The products are plain
// GEMMs (the host runs them); these kernels do the elementwise steps, the
// residual ||Z_k Y_k - I||_F, the symmetrisation of Z^T H Z and Z rho Z^T,
// and the Mulliken charges with the overlap.
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

// Tile pair (bi, bj), bi <= bj, of 32 x 32: both read through LDS, averaged,
// written back (a diagonal tile with its own transpose).
__global__ __launch_bounds__(256) void k_symmetrize(double* __restrict__ A, int N) {
    __shared__ double P[32][33], Q[32][33];
    const int nb = (N + 31) / 32;
    const long long T = (long long)nb * (nb + 1) / 2;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (long long t = blockIdx.x; t < T; t += gridDim.x) {
        int bi = 0;
        long long off = 0;
        while (t >= off + (nb - bi)) { off += nb - bi; ++bi; }
        const int bj = bi + (int)(t - off);
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = bi * 32 + r, j = bj * 32 + tx;
            const int i2 = bj * 32 + r, j2 = bi * 32 + tx;
            P[r][tx] = (i < N && j < N) ? A[(size_t)i * N + j] : 0.0;
            Q[r][tx] = (i2 < N && j2 < N) ? A[(size_t)i2 * N + j2] : 0.0;
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = bi * 32 + r, j = bj * 32 + tx;
            const int i2 = bj * 32 + r, j2 = bi * 32 + tx;
            const double a = 0.5 * (P[r][tx] + Q[tx][r]);      // (A_ij + A_ji) / 2
            const double b = 0.5 * (Q[r][tx] + P[tx][r]);      // (A_i2j2 + A_j2i2) / 2
            if (i < N && j < N) A[(size_t)i * N + j] = a;
            if (bi != bj && i2 < N && j2 < N) A[(size_t)i2 * N + j2] = b;
        }
    }
}

// One wave per atom: its four rows in order.
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
hipError_t launch_symmetrize(double* A, int N, hipStream_t s) {
    const long long nb = (N + 31) / 32;
    const long long T = nb * (nb + 1) / 2;
    hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)(T < 4096 ? T : 4096)), dim3(256), 0, s, A, N);
    return hipGetLastError();
}
hipError_t launch_mulliken_overlap(const double* D, const double* S, int n_atoms, double z_val, double* q,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_mulliken_overlap, dim3((n_atoms + 3) / 4), dim3(256), 0, s, D, S, n_atoms, z_val, q);
    return hipGetLastError();
}

}  // namespace sp2
