// Tight-binding Hamiltonian, Coulomb potential, forces, energies and the
// XL-BOMD integrator kernels (FP64) for the orthogonal T_e = 0 formulation.
//
// Model (SCC-TB subsection): two-centre Slater-Koster sp Hamiltonian h with
// radial bond integrals, quintic cut-off tail, gamma_ij = k_e / R_ij (i != j)
// and gamma_ii = U, H[n] = h + diag(V), V = gamma n (Eq. DFTB_2, S = I).
// All pair loops are brute force over atom pairs: at up to a few thousand
// atoms they are microseconds next to the density-matrix construction.
#include "tb_internal.h"

namespace sp2 {

__device__ __forceinline__ double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Radial function with tail: value and derivative.
__device__ __forceinline__ void radial(const Radial& f, double r, double& v, double& dv) {
    if (r < f.r1) {
        v = f.amp * exp(-(r - f.r0) / f.decay);
        dv = -v / f.decay;
    } else if (r < f.rcut) {
        const double x = r - f.r1;
        v = f.B[0] + x * (f.B[1] + x * (f.B[2] + x * (f.B[3] + x * (f.B[4] + x * f.B[5]))));
        dv = f.B[1] + x * (2.0 * f.B[2] + x * (3.0 * f.B[3] + x * (4.0 * f.B[4] + x * 5.0 * f.B[5])));
    } else {
        v = 0.0;
        dv = 0.0;
    }
}

// Slater-Koster block for unit vector c (atom i -> atom j) and magnitude t:
// ss = -t, s-p_k = c_k t, p_k-s = -c_k t, p_k-p_l = c_k c_l (2t) - delta_kl t
// (V_ss_sigma = -t, V_sp_sigma = t, V_pp_sigma = t, V_pp_pi = -t).
__device__ __forceinline__ void sk_block(const double c[3], double t, double B[4][4]) {
    B[0][0] = -t;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        B[0][k + 1] = c[k] * t;
        B[k + 1][0] = -c[k] * t;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const double cc = c[k] * c[l];   // symmetric in (k, l), so H is exactly symmetric
            B[k + 1][l + 1] = (2.0 * t) * cc - (k == l ? t : 0.0);
        }
    }
}

// g_x = sum_ab W[a][b] dB_ab/dd_x for the block B = sk_block(c, t(r)) of the
// pair vector d (|d| = r, c = d / r, dt = t'(r)): direction-cosine part
// dc_m/dd_x = (delta_mx - c_m c_x)/r and radial part dt/dd_x = dt c_x.
__device__ __forceinline__ void sk_grad_dot(const double c[3], double r, double t, double dt, const double W[4][4],
                                            double g[3]) {
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        double dc[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) dc[m] = ((m == x ? 1.0 : 0.0) - c[m] * c[x]) / r;
        const double dtt = dt * c[x];
        double s = -dtt * W[0][0];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const double dsp = dc[m] * t + c[m] * dtt;   // d(c_m t)
            s += dsp * (W[0][m + 1] - W[m + 1][0]);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const double dpp = 2.0 * (dtt * c[m] * c[l] + t * (dc[m] * c[l] + c[m] * dc[l]))
                                   - (m == l ? dtt : 0.0);
                s += dpp * W[m + 1][l + 1];
            }
        }
        g[x] = s;
    }
}

// V_i = sum_l gamma_il n_l: one wave per atom i.
__global__ __launch_bounds__(256) void k_potential(const double* __restrict__ xyz, const double* __restrict__ n,
                                                   int nat, double U, double ke, double* __restrict__ V) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nat) return;
    const double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2];
    double s = 0.0;
    for (int l = lane; l < nat; l += 64) {
        if (l == i) {
            s += U * n[l];
        } else {
            const double dx = xyz[3 * l] - xi, dy = xyz[3 * l + 1] - yi, dz = xyz[3 * l + 2] - zi;
            s += ke * n[l] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    }
    s = wsum(s);
    if (lane == 0) V[i] = s;
}

// H block row of atom i: one thread per (i, j) writes the 4 x 4 block H_ij.
__global__ __launch_bounds__(256) void k_hamiltonian(const double* __restrict__ xyz, int nat, TBArgs a,
                                                     const double* __restrict__ V, double* __restrict__ H) {
    const int i = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= nat) return;
    const size_t N = 4 * (size_t)nat;
    double B[4][4];
    if (i == j) {
        const double v = V ? V[i] : 0.0;
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) B[p][q] = 0.0;
        B[0][0] = a.eps_s + v;
        B[1][1] = B[2][2] = B[3][3] = a.eps_p + v;
    } else {
        const double dx = xyz[3 * j] - xyz[3 * i], dy = xyz[3 * j + 1] - xyz[3 * i + 1],
                     dz = xyz[3 * j + 2] - xyz[3 * i + 2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        double t = 0.0, dt;
        if (r < a.hop.rcut) radial(a.hop, r, t, dt);
        const double c[3] = {dx / r, dy / r, dz / r};
        sk_block(c, t, B);
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        double* row = H + (4 * (size_t)i + p) * N + 4 * (size_t)j;
        *reinterpret_cast<double2*>(row) = make_double2(B[p][0], B[p][1]);
        *reinterpret_cast<double2*>(row + 2) = make_double2(B[p][2], B[p][3]);
    }
}

// Overlap of the non-orthogonal variant, laid out like H: identity blocks on
// the diagonal, and for each pair the Slater-Koster block of the overlap
// integrals s(r) with the sign pattern opposite to the hopping's (-sk_block).
__global__ __launch_bounds__(256) void k_overlap(const double* __restrict__ xyz, int nat, Radial ov,
                                                 double* __restrict__ S) {
    const int i = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= nat) return;
    const size_t N = 4 * (size_t)nat;
    double B[4][4];
    if (i == j) {
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) B[p][q] = p == q ? 1.0 : 0.0;
    } else {
        const double dx = xyz[3 * j] - xyz[3 * i], dy = xyz[3 * j + 1] - xyz[3 * i + 1],
                     dz = xyz[3 * j + 2] - xyz[3 * i + 2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        double s = 0.0, ds;
        if (r < ov.rcut) radial(ov, r, s, ds);
        const double c[3] = {dx / r, dy / r, dz / r};
        sk_block(c, s, B);
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) B[p][q] = -B[p][q];
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        double* row = S + (4 * (size_t)i + p) * N + 4 * (size_t)j;
        *reinterpret_cast<double2*>(row) = make_double2(B[p][0], B[p][1]);
        *reinterpret_cast<double2*>(row + 2) = make_double2(B[p][2], B[p][3]);
    }
}

// Non-orthogonal charge shift: H_ab += (S_ab / 2)(V_atom(a) + V_atom(b)).
__global__ __launch_bounds__(256) void k_overlap_shift(double* __restrict__ H, const double* __restrict__ S,
                                                       const double* __restrict__ V, int nat) {
    const size_t N = 4 * (size_t)nat, n2 = N * N;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 256) {
        const size_t a = e / N, b = e % N;
        H[e] += 0.5 * S[e] * (V[a >> 2] + V[b >> 2]);
    }
}

// M = 2 W - (V_atom(a) + V_atom(b)) D_ab in place of W (W = D H D).
__global__ __launch_bounds__(256) void k_force_matrix(double* __restrict__ W, const double* __restrict__ D,
                                                      const double* __restrict__ V, int nat) {
    const size_t N = 4 * (size_t)nat, n2 = N * N;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 256) {
        const size_t a = e / N, b = e % N;
        W[e] = 2.0 * W[e] - (V[a >> 2] + V[b >> 2]) * D[e];
    }
}

// Overlap term of the non-orthogonal force: F_k += 2 sum_j sum_ab M_{ka,jb}
// d sk_block(c_kj, s(r_kj))_ab / d(R_j - R_k) (the overlap block is
// -sk_block with the overlap's radial function s); one wave per atom k.
__global__ __launch_bounds__(256) void k_forces_overlap(const double* __restrict__ xyz, int nat, Radial ov,
                                                        const double* __restrict__ M, double* __restrict__ F) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= nat) return;
    const size_t N = 4 * (size_t)nat;
    const double xk = xyz[3 * k], yk = xyz[3 * k + 1], zk = xyz[3 * k + 2];
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int j = lane; j < nat; j += 64) {
        if (j == k) continue;
        const double dx = xyz[3 * j] - xk, dy = xyz[3 * j + 1] - yk, dz = xyz[3 * j + 2] - zk;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r >= ov.rcut) continue;
        double s, ds;
        radial(ov, r, s, ds);
        const double c[3] = {dx / r, dy / r, dz / r};
        double Mkj[4][4];
        const double* Mp = M + 4 * (size_t)k * N + 4 * (size_t)j;
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) Mkj[p][qq] = Mp[p * N + qq];
        double g[3];
        sk_grad_dot(c, r, s, ds, Mkj, g);
        fx += 2.0 * g[0];
        fy += 2.0 * g[1];
        fz += 2.0 * g[2];
    }
    fx = wsum(fx);
    fy = wsum(fy);
    fz = wsum(fz);
    if (lane == 0) {
        F[3 * k] += fx;
        F[3 * k + 1] += fy;
        F[3 * k + 2] += fz;
    }
}

// Forces and per-atom energy terms at constant n; one wave per atom k.
//   F_k = 4 sum_j sum_ab D_{ka,jb} dB_kj/d(R_j - R_k)          (band)
//       - sum_j (q_k n_j + q_j n_k - n_k n_j) k_e (R_j - R_k)/r^3 (Coulomb)
//       + sum_j phi'(r) (R_j - R_k)/r                             (pair)
//   e_k = 2 sum_j sum_ab D_{ka,jb} h_{ka,jb} + q_k V_k - n_k V_k / 2
//         + 1/2 sum_j phi(r_kj)
__global__ __launch_bounds__(256) void k_forces(const double* __restrict__ xyz, int nat, TBArgs a,
                                                const double* __restrict__ D, const double* __restrict__ q,
                                                const double* __restrict__ n, const double* __restrict__ V,
                                                double* __restrict__ F, double* __restrict__ e_atom) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= nat) return;
    const size_t N = 4 * (size_t)nat;
    const double xk = xyz[3 * k], yk = xyz[3 * k + 1], zk = xyz[3 * k + 2];
    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
    for (int j = lane; j < nat; j += 64) {
        if (j == k) {
            // on-site part of 2 Tr[D h]
            const double* Dk = D + 4 * (size_t)k * N + 4 * (size_t)k;
            e += 2.0 * (a.eps_s * Dk[0] + a.eps_p * (Dk[N + 1] + Dk[2 * N + 2] + Dk[3 * N + 3]));
            continue;
        }
        const double dx = xyz[3 * j] - xk, dy = xyz[3 * j + 1] - yk, dz = xyz[3 * j + 2] - zk;
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double r = sqrt(r2);
        const double d[3] = {dx, dy, dz};
        // Coulomb
        const double w = q[k] * n[j] + q[j] * n[k] - n[k] * n[j];
        const double cw = w * a.coulomb_k / (r2 * r);
        fx -= cw * dx;
        fy -= cw * dy;
        fz -= cw * dz;
        if (r >= a.hop.rcut) continue;
        // pair
        double ph, dph;
        radial(a.pair, r, ph, dph);
        if (a.pair.amp != 0.0) {
            e += 0.5 * ph;
            fx += dph * dx / r;
            fy += dph * dy / r;
            fz += dph * dz / r;
        }
        // band
        double t, dt;
        radial(a.hop, r, t, dt);
        const double c[3] = {dx / r, dy / r, dz / r};
        double Dkj[4][4];
        const double* Dp = D + 4 * (size_t)k * N + 4 * (size_t)j;
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) Dkj[p][qq] = Dp[p * N + qq];
        double B[4][4];
        sk_block(c, t, B);
        double eb = 0.0;
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) eb += Dkj[p][qq] * B[p][qq];
        e += 2.0 * eb;
        double g[3];
        sk_grad_dot(c, r, t, dt, Dkj, g);
        fx += 4.0 * g[0];
        fy += 4.0 * g[1];
        fz += 4.0 * g[2];
    }
    fx = wsum(fx);
    fy = wsum(fy);
    fz = wsum(fz);
    e = wsum(e);
    if (lane == 0) {
        if (F) {
            F[3 * k] = fx;
            F[3 * k + 1] = fy;
            F[3 * k + 2] = fz;
        }
        e_atom[k] = e + q[k] * V[k] - 0.5 * n[k] * V[k];
    }
}

// Fixed-order sum of x[0..n) into *out (one workgroup).
__global__ __launch_bounds__(256) void k_sum(const double* __restrict__ x, int n, double* __restrict__ out) {
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) s += x[k];
    s = wsum(s);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Velocity Verlet half kick (and optional drift): v += h a_conv F; x += dt v.
__global__ void k_kick_drift(double* __restrict__ x, double* __restrict__ v, const double* __restrict__ F,
                             int n3, double half_dt_acc, double dt) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n3) return;
    const double vv = v[e] + half_dt_acc * F[e];
    v[e] = vv;
    if (dt != 0.0) x[e] += dt * vv;
}

// Eq. Verl_n: n_new = 2 n_t - n_{t-dt} + kappa (q_t - n_t) + alpha sum_k c_k n_{t-k dt}.
// hist holds K+1 rows of nat values; row (head + k) mod (K+1) is n_{t-k dt}.
// Writes n_new into row (head + K) mod (K+1) (the oldest, no longer needed
// after this step).
__global__ void k_xl_charges(double* __restrict__ hist, int nat, int K, int head, const double* __restrict__ q,
                             XLArgs a) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nat) return;
    const int L = K + 1;
    const double nt = hist[(size_t)head * nat + i];
    const double ntm1 = hist[(size_t)((head + 1) % L) * nat + i];
    double diss = 0.0;
    for (int k = 0; k <= K; ++k) diss += a.c[k] * hist[(size_t)((head + k) % L) * nat + i];
    const double nn = 2.0 * nt - ntm1 + a.kappa * (q[i] - nt) + a.alpha * diss;
    hist[(size_t)((head + K) % L) * nat + i] = nn;
}

__global__ void k_absdiff(const double* __restrict__ a, const double* __restrict__ b, int n,
                          double* __restrict__ d) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) d[i] = fabs(a[i] - b[i]);
}

// Linear charge mixing n += beta (q - n).
__global__ void k_mix(double* __restrict__ n, const double* __restrict__ q, int nat, double beta) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < nat) n[i] += beta * (q[i] - n[i]);
}

__global__ void k_max(const double* __restrict__ x, int n, double* __restrict__ out) {
    double m = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) m = fmax(m, x[k]);
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) *out = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__global__ void k_sqsum3(const double* __restrict__ v, int n3, double* __restrict__ part) {
    double s = 0.0;
    for (int e = threadIdx.x; e < n3; e += 256) s += v[e] * v[e];
    s = wsum(s);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *part = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// ------------------------------------------------------------------ launch
hipError_t launch_potential(const double* xyz, const double* n, int nat, double U, double ke, double* V,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_potential, dim3((nat + 3) / 4), dim3(256), 0, s, xyz, n, nat, U, ke, V);
    return hipGetLastError();
}
hipError_t launch_hamiltonian(const double* xyz, int nat, const TBArgs& a, const double* V, double* H,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_hamiltonian, dim3((nat + 255) / 256, nat), dim3(256), 0, s, xyz, nat, a, V, H);
    return hipGetLastError();
}
static int grid_n2(int nat) {
    const size_t n2 = 16 * (size_t)nat * nat, g = (n2 + 255) / 256;
    return (int)(g < 4096 ? g : 4096);
}
hipError_t launch_overlap_shift(double* H, const double* S, const double* V, int nat, hipStream_t s) {
    hipLaunchKernelGGL(k_overlap_shift, dim3(grid_n2(nat)), dim3(256), 0, s, H, S, V, nat);
    return hipGetLastError();
}
hipError_t launch_force_matrix(double* W, const double* D, const double* V, int nat, hipStream_t s) {
    hipLaunchKernelGGL(k_force_matrix, dim3(grid_n2(nat)), dim3(256), 0, s, W, D, V, nat);
    return hipGetLastError();
}
hipError_t launch_forces_overlap(const double* xyz, int nat, const Radial& ov, const double* M, double* F,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_forces_overlap, dim3((nat + 3) / 4), dim3(256), 0, s, xyz, nat, ov, M, F);
    return hipGetLastError();
}
hipError_t launch_overlap(const double* xyz, int nat, const Radial& ov, double* S, hipStream_t s) {
    hipLaunchKernelGGL(k_overlap, dim3((nat + 255) / 256, nat), dim3(256), 0, s, xyz, nat, ov, S);
    return hipGetLastError();
}
hipError_t launch_forces(const double* xyz, int nat, const TBArgs& a, const double* D, const double* q,
                         const double* n, const double* V, double* F, double* e_atom, double* e_out,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_forces, dim3((nat + 3) / 4), dim3(256), 0, s, xyz, nat, a, D, q, n, V, F, e_atom);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, e_atom, nat, e_out);
    return hipGetLastError();
}
hipError_t launch_kick_drift(double* x, double* v, const double* F, int n3, double half_dt_acc, double dt,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_kick_drift, dim3((n3 + 255) / 256), dim3(256), 0, s, x, v, F, n3, half_dt_acc, dt);
    return hipGetLastError();
}
hipError_t launch_xl_charges(double* hist, int nat, int K, int head, const double* q, const XLArgs& a,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_xl_charges, dim3((nat + 255) / 256), dim3(256), 0, s, hist, nat, K, head, q, a);
    return hipGetLastError();
}
hipError_t launch_maxdiff(const double* a, const double* b, int n, double* tmp, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_absdiff, dim3((n + 255) / 256), dim3(256), 0, s, a, b, n, tmp);
    hipLaunchKernelGGL(k_max, dim3(1), dim3(256), 0, s, tmp, n, out);
    return hipGetLastError();
}
hipError_t launch_mix(double* n, const double* q, int nat, double beta, hipStream_t s) {
    hipLaunchKernelGGL(k_mix, dim3((nat + 255) / 256), dim3(256), 0, s, n, q, nat, beta);
    return hipGetLastError();
}
hipError_t launch_sqsum(const double* v, int n3, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sqsum3, dim3(1), dim3(256), 0, s, v, n3, out);
    return hipGetLastError();
}

}  // namespace sp2
