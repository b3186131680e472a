/* Oracle (test infrastructure only): cyclic Jacobi eigensolver for a dense
 * real symmetric matrix, FP64, no LAPACK.
 *
 * It provides the plain definition of the zero-temperature density matrix
 * theta(mu0 I - H) used in the orthogonal T_e = 0 formulation (the step
 * function of the Hamiltonian): eigenvectors of H, filled in ascending order.
 *
 * Method: the classical two-sided Jacobi rotation (Golub & Van Loan,
 * "Matrix Computations", section 8.5, the symmetric Schur decomposition of a
 * 2x2 block followed by A <- J^T A J), swept cyclically row by row over all
 * pairs p < q until off(A) <= tol * ||A||_F.
 *
 * Pinned by closed forms (diagonal and 2x2 matrices) and against an
 * independent library eigensolver in tests/test_oracle_eig.py.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

static double off_norm(int n, const double *a)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j) s += a[(size_t)i * n + j] * a[(size_t)i * n + j];
    return sqrt(s);
}

static double frob_norm(int n, const double *a)
{
    double s = 0.0;
    for (size_t k = 0; k < (size_t)n * n; ++k) s += a[k] * a[k];
    return sqrt(s);
}

/* Eigen-decomposition A = V diag(w) V^T.
 *   n      matrix order
 *   a      n*n row-major symmetric input; overwritten (ends near-diagonal)
 *   w      out: n eigenvalues (unsorted, diagonal of the final A)
 *   v      out: n*n row-major; column k is the eigenvector of w[k]
 *   tol    relative stopping tolerance on off(A)/||A||_F
 *   max_sweeps  sweep limit
 * Returns the number of sweeps done, or -1 if the limit was reached. */
int oracle_jacobi_eigh(int n, double *a, double *w, double *v, double tol,
                       int max_sweeps)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) v[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;

    double fro = frob_norm(n, a);
    int sweep = 0;
    if (fro == 0.0) goto done;

    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        if (off_norm(n, a) <= tol * fro) goto done;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                double app = a[(size_t)p * n + p];
                double aqq = a[(size_t)q * n + q];
                /* 2x2 symmetric Schur: choose t = tan(theta), the smaller root */
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                        : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                /* A <- A J : columns p and q */
                for (int k = 0; k < n; ++k) {
                    double akp = a[(size_t)k * n + p];
                    double akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - s * akq;
                    a[(size_t)k * n + q] = s * akp + c * akq;
                }
                /* A <- J^T A : rows p and q */
                for (int k = 0; k < n; ++k) {
                    double apk = a[(size_t)p * n + k];
                    double aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - s * aqk;
                    a[(size_t)q * n + k] = s * apk + c * aqk;
                }
                a[(size_t)p * n + q] = 0.0;
                a[(size_t)q * n + p] = 0.0;
                /* V <- V J */
                for (int k = 0; k < n; ++k) {
                    double vkp = v[(size_t)k * n + p];
                    double vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = c * vkp - s * vkq;
                    v[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    if (off_norm(n, a) > tol * fro) {
        for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
        return -1;
    }
done:
    for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
    return sweep;
}
