"""Oracle: the finite electronic temperature density matrix, FP64.

Test infrastructure only.  At T_e > 0 the paper's density is the Fermi
operator of H (Eq. EL_4c; Eq. DM_perp for the orthogonalised H), f(H) =
(exp(beta (H - mu I)) + 1)^(-1), beta = 1 / (k_B T_e), built by the
recursive Fermi-operator expansion it cites.  Readings (the paper cites the
method without printing it, and leaves mu open):

* definition: f(H) = V diag(f_i) V^T from the eigen-decomposition of H,
  f_i = 1 / (1 + exp(beta (e_i - mu))), with mu the canonical chemical
  potential, sum_i f_i = N_occ (solved by bisection); the eigenpairs come
  from the oracle's own Jacobi solver (solver="jacobi", the default) or, for
  the few full-size comparisons where Jacobi is too slow (N > 600), from the
  library eigensolver (solver="lapack", named at the call);
* the inverse inside the recursion is a library primitive (numpy's inverse),
  taken as one step of the printed formula;
* the recursion: with y = beta (H - mu I) / 2^(n+2), X_0 = I/2 - y; then n
  times X_{k+1} = X_k^2 (X_k^2 + (I - X_k)^2)^(-1).  The ratio (I - X)/X
  squares at every step and starts at (I/2 + y)/(I/2 - y) ~ exp(4y), so X_n
  approaches (exp(beta (H - mu I)) + 1)^(-1): its exponent carries a relative
  error of about (4y)^2 / 12, i.e. (beta |e - mu| / 2^n)^2 / 12;
* energy at T_e > 0: the electronic entropy of the occupations f_i (the
  eigenvalues of D), S = -2 k_B sum_i [f_i ln f_i + (1 - f_i) ln(1 - f_i)]
  (Eq. Entropy), and the free energy A = U(R; n) - T_e S with U as at T_e = 0
  evaluated with the Fermi D.  D makes 2 Tr[D H[n]] - T_e S stationary at
  fixed N, so -dA/dR at constant n is the T_e = 0 force expression with the
  Fermi D (pinned by finite differences);
* mu for the recursion: Tr X_n grows monotonically with mu, so mu is solved
  by Newton steps on Tr X_n = N_occ with d Tr X_n / d mu ~ beta Tr[X_n (I -
  X_n)] (the derivative of the Fermi function), safeguarded by bisection: the
  root stays bracketed, starting from [e_min - 40 kT, e_max + 40 kT] (the
  Gershgorin bounds widened until every Fermi factor is below e^-40 at the
  lower end and above 1 - e^-40 at the upper), and a Newton step that leaves
  the bracket is replaced by its midpoint.  The first mu is the midpoint of the
  Gershgorin bounds.
"""
from __future__ import annotations

import numpy as np

from . import eig, observables, sp2, tb

KB_EV_PER_K = 8.617333262e-5


def fermi_occupations(e, mu, beta):
    x = np.clip(beta * (np.asarray(e) - mu), -700.0, 700.0)
    return 1.0 / (1.0 + np.exp(x))


def canonical_mu(e, n_occ, beta, tol=1e-14):
    """mu with sum_i f(e_i) = n_occ, by bisection."""
    lo, hi = float(np.min(e)) - 50.0 / beta, float(np.max(e)) + 50.0 / beta
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if fermi_occupations(e, mid, beta).sum() > n_occ:
            hi = mid
        else:
            lo = mid
        if hi - lo < tol:
            break
    return 0.5 * (lo + hi)


def eigenpairs(A, solver="jacobi"):
    """Ascending eigenvalues and eigenvectors (columns) of symmetric A."""
    if solver == "jacobi":
        return eig.jacobi_eigh(A)
    if solver == "lapack":
        return np.linalg.eigh(A)
    raise ValueError(solver)


def fermi_density(H, n_occ, kT, solver="jacobi"):
    """(D, mu, occupations) of the definition (kT in eV)."""
    beta = 1.0 / kT
    e, V = eigenpairs(H, solver)
    mu = canonical_mu(e, n_occ, beta)
    f = fermi_occupations(e, mu, beta)
    return (V * f) @ V.T, mu, f


def recursive_fermi(H, mu, kT, n_steps):
    """X_n of the recursive expansion at chemical potential mu."""
    N = H.shape[0]
    y = (H - mu * np.eye(N)) / (kT * 2.0 ** (n_steps + 2))
    X = 0.5 * np.eye(N) - y
    for _ in range(n_steps):
        X2 = X @ X
        A = 2.0 * X2 - 2.0 * X + np.eye(N)        # X^2 + (I - X)^2
        X = X2 @ np.linalg.inv(A)
        X = 0.5 * (X + X.T)
    return X


def recursive_fermi_canonical(H, n_occ, kT, n_steps, tol=1e-10, max_newton=100):
    """(X_n, mu, passes) with |Tr X_n - n_occ| < tol."""
    beta = 1.0 / kT
    e_lo, e_hi = sp2.gershgorin(H)
    lo, hi = e_lo - 40.0 * kT, e_hi + 40.0 * kT
    mu = 0.5 * (e_lo + e_hi)
    for it in range(max_newton):
        X = recursive_fermi(H, mu, kT, n_steps)
        t = float(np.trace(X))
        if abs(t - n_occ) < tol:
            return X, mu, it + 1
        if t < n_occ:
            lo = mu
        else:
            hi = mu
        d = beta * (t - float(np.sum(X * X)))
        step = mu - (t - n_occ) / d if d > 0.0 else np.nan
        mu = step if lo < step < hi else 0.5 * (lo + hi)
    raise RuntimeError("Newton on mu did not converge")


def entropy(f):
    """S / k_B of occupations f (Eq. Entropy; the factor 2 counts spin)."""
    f = np.asarray(f, dtype=np.float64)
    s = np.zeros_like(f)
    inner = (f > 0.0) & (f < 1.0)
    g = f[inner]
    s[inner] = g * np.log(g) + (1.0 - g) * np.log1p(-g)
    return -2.0 * float(s.sum())


def free_energy(pos, n, m, n_occ, kT, solver="jacobi"):
    """(A, D, mu): A = U(R; n) - kT S / k_B with D the canonical Fermi operator of H[n]."""
    H = tb.hamiltonian(pos, n, m)
    D, mu, f = fermi_density(H, n_occ, kT, solver)
    return observables.potential_energy(pos, n, D, m) - kT * entropy(f), D, mu
