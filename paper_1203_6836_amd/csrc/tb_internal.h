// Internal declarations of the tight-binding / force / XL-BOMD kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace sp2 {

// amp * exp(-(r - r0)/decay) for r < r1; sum_k B_k (r - r1)^k on [r1, rcut); 0 beyond.
struct Radial {
    double amp, r0, decay, r1, rcut;
    double B[6];
};

struct TBArgs {
    double eps_s, eps_p;
    double hubbard_u, coulomb_k;
    Radial hop;
    Radial pair;
};

struct XLArgs {
    double kappa, alpha;
    double c[9];
};

hipError_t launch_potential(const double* xyz, const double* n, int nat, double U, double ke, double* V,
                            hipStream_t s);
hipError_t launch_hamiltonian(const double* xyz, int nat, const TBArgs& a, const double* V, double* H,
                              hipStream_t s);
// Non-orthogonal charge shift H += (S L + L S)/2 (V per atom); the force
// matrix M = 2 W - (V_a + V_b) D in place of W = D H D; the overlap term of
// the force added to F.
hipError_t launch_overlap_shift(double* H, const double* S, const double* V, int nat, hipStream_t s);
hipError_t launch_force_matrix(double* W, const double* D, const double* V, int nat, hipStream_t s);
hipError_t launch_forces_overlap(const double* xyz, int nat, const Radial& ov, const double* M, double* F,
                                 hipStream_t s);
// S of the non-orthogonal variant for overlap radial function ov.
hipError_t launch_overlap(const double* xyz, int nat, const Radial& ov, double* S, hipStream_t s);
hipError_t launch_forces(const double* xyz, int nat, const TBArgs& a, const double* D, const double* q,
                         const double* n, const double* V, double* F, double* e_atom, double* e_out,
                         hipStream_t s);
hipError_t launch_kick_drift(double* x, double* v, const double* F, int n3, double half_dt_acc, double dt,
                             hipStream_t s);
hipError_t launch_xl_charges(double* hist, int nat, int K, int head, const double* q, const XLArgs& a,
                             hipStream_t s);
hipError_t launch_maxdiff(const double* a, const double* b, int n, double* tmp, double* out, hipStream_t s);
hipError_t launch_mix(double* n, const double* q, int nat, double beta, hipStream_t s);
hipError_t launch_sqsum(const double* v, int n3, double* out, hipStream_t s);

}  // namespace sp2
