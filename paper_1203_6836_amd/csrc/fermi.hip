// Finite electronic temperature (Eq. EL_4c's Fermi operator, recursive
// Fermi-operator expansion): with y = beta (H - mu I) / 2^(n+2), X_0 = I/2 - y
// and n steps X_{k+1} = X_k^2 (X_k^2 + (I - X_k)^2)^(-1) give
// (exp(beta (H - mu I)) + 1)^(-1) (the ratio (I - X)/X squares each step).
// The products run in the FP64 product kernel; these kernels form X_0, A = X^2 + (I - X)^2, the
// Newton-Schulz steps of A^(-1) (A = I/2 + 2 (X - I/2)^2 has its spectrum in
// [1/2, 1] while X has its own in [0, 1], and nearer 1/2 in the first steps),
// and the trace and Frobenius sums of the Newton step on mu.
#include "fermi_internal.h"

namespace sp2 {

__device__ __forceinline__ double wsum_f(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double block_sum(double v, double* sw) {
    v = wsum_f(v);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (sw[0] + sw[1]) + (sw[2] + sw[3]);
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_fermi_init(const double* __restrict__ H, int N, double mu, double scale,
                                                    double* __restrict__ X) {
    const size_t n2 = (size_t)N * N;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 256) {
        const size_t i = e / N, j = e % N;
        X[e] = (i == j ? 0.5 : 0.0) - (H[e] - (i == j ? mu : 0.0)) * scale;
    }
}

__global__ __launch_bounds__(256) void k_fermi_a(const double* __restrict__ X2, const double* __restrict__ X, int N,
                                                 double c, double* __restrict__ A, double* __restrict__ Y) {
    const size_t n2 = (size_t)N * N;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 256) {
        const double d = (e / N == e % N) ? 1.0 : 0.0;
        const double a = 2.0 * X2[e] - 2.0 * X[e] + d;
        A[e] = a;
        Y[e] = c * (2.0 * d - c * a);
    }
}

__global__ __launch_bounds__(256) void k_trace_fro(const double* __restrict__ X, int N, double* __restrict__ part) {
    __shared__ double sw[4];
    const size_t n2 = (size_t)N * N;
    double tr = 0.0, fr = 0.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 256) {
        const double x = X[e];
        if (e / N == e % N) tr += x;
        fr += x * x;
    }
    tr = block_sum(tr, sw);
    fr = block_sum(fr, sw);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = tr;
        part[2 * blockIdx.x + 1] = fr;
    }
}

__global__ __launch_bounds__(256) void k_sum_pairs(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double sw[4];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    a = block_sum(a, sw);
    b = block_sum(b, sw);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

__global__ __launch_bounds__(256) void k_cheb_init(const double* __restrict__ H, int N, double c, double inv_w,
                                                   double* __restrict__ Ht, double* __restrict__ T0) {
    const size_t n2 = (size_t)N * N;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 256) {
        const bool d = e / N == e % N;
        Ht[e] = (H[e] - (d ? c : 0.0)) * inv_w;
        T0[e] = d ? 1.0 : 0.0;
    }
}

static int grid_elem(int N) {
    const size_t g = ((size_t)N * N + 255) / 256;
    return (int)(g < 4096 ? g : 4096);
}

hipError_t launch_fermi_init(const double* H, int N, double mu, double scale, double* X, hipStream_t s) {
    hipLaunchKernelGGL(k_fermi_init, dim3(grid_elem(N)), dim3(256), 0, s, H, N, mu, scale, X);
    return hipGetLastError();
}
hipError_t launch_fermi_a(const double* X2, const double* X, int N, double c, double* A, double* Y, hipStream_t s) {
    hipLaunchKernelGGL(k_fermi_a, dim3(grid_elem(N)), dim3(256), 0, s, X2, X, N, c, A, Y);
    return hipGetLastError();
}
hipError_t launch_cheb_init(const double* H, int N, double c, double inv_w, double* Ht, double* T0, hipStream_t s) {
    hipLaunchKernelGGL(k_cheb_init, dim3(grid_elem(N)), dim3(256), 0, s, H, N, c, inv_w, Ht, T0);
    return hipGetLastError();
}
hipError_t launch_trace_fro(const double* X, int N, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_trace_fro, dim3(kFermiBlocks), dim3(256), 0, s, X, N, part);
    return hipGetLastError();
}
hipError_t launch_sum_pairs(const double* part, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}

}  // namespace sp2
