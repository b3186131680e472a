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
  symmetric one, is used (then rho does not depend on the choice);
* charges: Mulliken, q_i = 2 sum_{alpha in i} (rho S)_{i alpha, i alpha} - z_i.
  The paper names them Mulliken charges and differentiates them as
  2 sum (rho S_R) (the charge-derivative equation), which is the derivative
  of these; its printed charge formula, with the diagonal of rho_perp, would
  give Loewdin charges for Z = S^(-1/2).
"""
from __future__ import annotations

import numpy as np

from . import sp2, tb


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


def loewdin_factor(S):
    """Z = S^(-1/2) from the eigen-decomposition of S (Z^T S Z = I)."""
    w, V = np.linalg.eigh(S)
    return (V / np.sqrt(w)) @ V.T


def density_matrix(H, S, n_occ, **sp2_kw):
    """(rho, rho_perp, Z, SP2 result): SP2 of H_perp = Z^T H Z, then
    rho = Z rho_perp Z^T."""
    Z = loewdin_factor(S)
    Hp = Z.T @ H @ Z
    Hp = 0.5 * (Hp + Hp.T)
    r = sp2.sp2(Hp, n_occ, **sp2_kw)
    rho = Z @ r.D @ Z.T
    return rho, r.D, Z, r


def mulliken(rho, S, z_val=4):
    """Net Mulliken charges 2 sum_{alpha in i} (rho S)_{alpha alpha} - z_val."""
    pop = np.einsum("ab,ba->a", rho, S)
    return 2.0 * pop.reshape(-1, 4).sum(axis=1) - z_val
