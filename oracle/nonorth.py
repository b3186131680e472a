"""Oracle: the non-orthogonal formulation (density matrix and charges), FP64.

Test infrastructure only.  The paper's non-orthogonal self-consistent
tight-binding (Non-orthogonal formulation subsection) orthogonalises the
Hamiltonian with a congruence factor Z, Z^T S Z = I (Eq. Congr), as
H_perp = Z^T H Z, takes the density matrix of H_perp (Eq. DM_perp; at
T_e = 0 the step function theta(mu0 I - H_perp) of the orthogonal case), and
de-orthogonalises it as rho = Z rho_perp Z^T.

Readings (the paper leaves these open):
* the overlap of the synthetic sp model (LATTE's parameters are not given):
  S = I plus, for every pair closer than r_cut, the 4 x 4 Slater-Koster
  block of overlap integrals of magnitude s(r) = s0 exp(-(r - r0)/lambda_s)
  with the hopping's tail, with the sign pattern opposite to the hopping's
  (overlap and hopping of a bonding pair have opposite signs);
* Z: any congruence factor is allowed; the Loewdin factor S^(-1/2), the
  symmetric one, is used (then rho does not depend on the choice), from the
  eigenpairs of S by the oracle's Jacobi solver (solver="jacobi", the
  default) or, for the comparisons at N > 600, the library eigensolver
  (solver="lapack", named at the call);
* charges: Mulliken, q_i = 2 sum_{alpha in i} (rho S)_{i alpha, i alpha} - z_i.
  The paper names them Mulliken charges and differentiates them as
  2 sum (rho S_R) (the charge-derivative equation), which is the derivative
  of these; its printed charge formula, with the diagonal of rho_perp, would
  give Loewdin charges for Z = S^(-1/2).

Energy and forces at constant auxiliary charges n, written for the overlap
the way the orthogonal oracle writes them (observables module):
* H[n] = h + (S L + L S) / 2, L the diagonal of V_i = (gamma n)_i on the
  orbitals of atom i (the charge shift of a non-orthogonal basis);
* U(R; n) = 2 Tr[rho h] + sum_i q_i V_i - 1/2 n^T gamma n + E_pair, q the
  Mulliken charges above (equal to 2 Tr[rho H] - z sum_i V_i - 1/2 n^T gamma n
  + E_pair);
* F_k = -dU/dR_k.  rho is the generalized projector of H[n] (H c = e S c),
  so the generalized Hellmann-Feynman theorem removes d rho and adds the
  energy-weighted term -2 Tr[W dS/dR_k], W = rho H rho; the S inside H[n]
  and inside q add (V_a + V_b) rho_ab dS_ab/dR_k.  Result: the orthogonal
  force with these charges, plus sum_ab M_ab dS_ab/dR_k with
  M = 2 W - (V_a + V_b) rho_ab (a, b orbital indices; V of their atoms).
  This is the role of the Pulay term Tr[(S^-1 H rho + rho H S^-1) S_R] and
  of the charge-derivative term of the paper's non-orthogonal force equation
  (at T_e = 0 and idempotent rho, W = rho H rho).  Pinned by central finite
  differences of U with rho recomputed at each displaced geometry.

Finite electronic temperature in this basis (the non-orthogonal free energy
with the entropy term of the Non-orthogonal formulation subsection): rho =
Z f(H_perp) Z^T with f the Fermi function at the canonical mu (Tr[rho S] =
n_occ), the free energy U - T_e S of the entropy of the occupations (Eq.
Entropy), and the forces of the free energy: the generalized
Hellmann-Feynman theorem for Fermi occupations gives the same expression
with the energy-weighted W = Z f(H_perp) H_perp Z^T in place of rho H rho
(they differ when rho is not idempotent).  Pinned by central finite
differences of the free energy with rho and mu recomputed at each displaced
geometry.
"""
from __future__ import annotations

import numpy as np

from . import eig, fermi, observables, sp2, tb


def overlap(pos, m):
    """S (N x N, N = 4 n_atoms) of model m (fields overlap_s0, overlap_lam)."""
    nat = len(pos)
    N = 4 * nat
    S = np.eye(N)
    if m.overlap_s0 == 0.0:
        return S
    ii, jj, d, r = tb.neighbour_pairs(pos, m.r_cut)
    s, _ = tb.radial(r, m.overlap_s0, m.r0, m.overlap_lam, m.r_tail, m.r_cut)
    for a, b, dv, rv, sv in zip(ii, jj, d, r, s):
        B = -tb.sk_block(dv / rv, sv)
        S[4 * a:4 * a + 4, 4 * b:4 * b + 4] = B
        S[4 * b:4 * b + 4, 4 * a:4 * a + 4] = B.T
    return S


def loewdin_factor(S, solver="jacobi"):
    """Z = S^(-1/2) from the eigen-decomposition of S (Z^T S Z = I)."""
    if solver == "jacobi":
        w, V = eig.jacobi_eigh(S)
    elif solver == "lapack":
        w, V = np.linalg.eigh(S)
    else:
        raise ValueError(solver)
    return (V / np.sqrt(w)) @ V.T


def density_matrix(H, S, n_occ, solver="jacobi", **sp2_kw):
    """(rho, rho_perp, Z, SP2 result): SP2 of H_perp = Z^T H Z, then
    rho = Z rho_perp Z^T (solver: how the Loewdin factor is formed)."""
    Z = loewdin_factor(S, solver)
    Hp = Z.T @ H @ Z
    Hp = 0.5 * (Hp + Hp.T)
    r = sp2.sp2(Hp, n_occ, **sp2_kw)
    rho = Z @ r.D @ Z.T
    return rho, r.D, Z, r


def mulliken(rho, S, z_val=4):
    """Net Mulliken charges 2 sum_{alpha in i} (rho S)_{alpha alpha} - z_val."""
    pop = np.einsum("ab,ba->a", rho, S)
    return 2.0 * pop.reshape(-1, 4).sum(axis=1) - z_val


def potential(pos, n, m):
    """V_i = (gamma n)_i repeated on the four orbitals of each atom."""
    return np.repeat(tb.onsite_potential(pos, np.asarray(n, dtype=np.float64), m), 4)


def hamiltonian(pos, n, m, S=None):
    """H[n] = h + (S L + L S) / 2 (h alone for n = None)."""
    h = tb.hamiltonian0(pos, m)
    if n is None:
        return h
    S = overlap(pos, m) if S is None else S
    v = potential(pos, n, m)
    return h + 0.5 * S * (v[:, None] + v[None, :])


def potential_energy(pos, n, rho, m, S=None):
    S = overlap(pos, m) if S is None else S
    q = mulliken(rho, S, m.z_val)
    g = tb.gamma_matrix(pos, m)
    h = tb.hamiltonian0(pos, m)
    return 2.0 * float(np.sum(rho * h)) + observables.coulomb_energy(q, n, g) + tb.pair_energy(pos, m)


def overlap_block_grad(dv, m):
    """d S_ij / d(R_j - R_i) of one pair block, shape (3, 4, 4): the gradient of
    -sk_block with the overlap's radial function."""
    ms = m.with_(t0=m.overlap_s0, lam=m.overlap_lam)
    return -tb.sk_block_grad(dv, ms)


def forces(pos, n, rho, m, S=None, W=None):
    """F_k = -dU/dR_k at constant n; shape (n_atoms, 3).  W: the
    energy-weighted density matrix (default rho H rho, the T_e = 0 form)."""
    S = overlap(pos, m) if S is None else S
    q = mulliken(rho, S, m.z_val)
    F = observables.forces(pos, n, rho, m, q=q)
    H = hamiltonian(pos, n, m, S)
    v = potential(pos, n, m)
    W = rho @ H @ rho if W is None else W
    M = 2.0 * W - (v[:, None] + v[None, :]) * rho
    ii, jj, d, r = tb.neighbour_pairs(pos, m.r_cut)
    for a, b, dv in zip(ii, jj, d):
        G = overlap_block_grad(dv, m)
        g = 2.0 * np.einsum("xij,ij->x", G, M[4 * a:4 * a + 4, 4 * b:4 * b + 4])
        F[b] += g
        F[a] -= g
    return F


def fermi_density_matrix(H, S, n_occ, kT, solver="jacobi"):
    """(rho, W, mu, f): the Fermi operator of the generalized eigenproblem
    H c = e S c at the canonical mu (kT in eV): rho = Z f(H_perp) Z^T, and
    the energy-weighted W = Z f(H_perp) H_perp Z^T, from the eigenpairs of
    H_perp = Z^T H Z (Z the Loewdin factor; solver as in loewdin_factor)."""
    Z = loewdin_factor(S, solver)
    Hp = Z.T @ H @ Z
    e, V = fermi.eigenpairs(0.5 * (Hp + Hp.T), solver)
    beta = 1.0 / kT
    mu = fermi.canonical_mu(e, n_occ, beta)
    f = fermi.fermi_occupations(e, mu, beta)
    C = Z @ V
    rho = (C * f) @ C.T
    W = (C * (f * e)) @ C.T
    return rho, W, mu, f


def free_energy(pos, n, m, n_occ, kT, solver="jacobi"):
    """(A, rho, W, mu): A = U(R; n) - kT S / k_B with rho the Fermi operator
    of H[n] in this basis."""
    S = overlap(pos, m)
    H = hamiltonian(pos, n, m, S)
    rho, W, mu, f = fermi_density_matrix(H, S, n_occ, kT, solver)
    return potential_energy(pos, n, rho, m, S) - kT * fermi.entropy(f), rho, W, mu
