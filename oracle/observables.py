"""Oracle: charges, energies and forces of the orthogonal T_e = 0 model.

Test infrastructure only.

* Mulliken charges (the net-charge equation after Eq. DFTB_2, S = I):
  q_i = 2 sum_{alpha in i} (rho - rho0)_{i alpha, i alpha}.  Reading: rho0 of
  the separate neutral atoms puts 2 electrons per spin channel on each atom
  (four valence electrons), so q_i = 2 sum_alpha rho_{i alpha,i alpha} - 4
  (electron excess; sum_i q_i = 2 (Tr rho - N_occ) = 0).
* band energy 2 Tr[rho H] = 2 sum of occupied eigenvalues (Eq. DFT_POT).
* potential energy: Eq. HF_POT_2 (Harris-Foulkes form, Eq. Approx) written
  for charges: U(R; n) = 2 Tr[rho h] + sum_i q_i V_i - 1/2 n^T gamma n + E_pair
  with V = gamma n, H[n] = h + diag(V) and rho = theta(mu0 I - H[n]).  At
  n = q this is the SCC-TB energy 2 Tr[rho h] + 1/2 q^T gamma q + E_pair
  (Eq. DFTB_1 with 2 sum eps = 2 Tr[rho H]).
* forces: F_k = -dU/dR_k at constant n.  Because rho minimises Tr[rho H[n]]
  at fixed trace, the d rho terms drop and
  F_k = -2 Tr[rho dh/dR_k] - sum_ij (q_i n_j - 1/2 n_i n_j) dgamma_ij/dR_k
        - dE_pair/dR_k.
  This is Eq. EL_Orth_a with Eq. EL_Orth_c, reading rho as rho - rho0 in
  the on-site gamma term (otherwise it is not the gradient of any energy of
  Eq. DFTB_1 form).  Pinned by central finite differences of U.
* total energy: E_tot = kinetic + U (Eq. EtotOrth with S = 0 at T_e = 0).
"""
from __future__ import annotations

import numpy as np

from . import tb


def mulliken(D, z_val=4):
    """Net Mulliken charges (electron excess) per atom from the N x N projector."""
    occ = np.diag(D).reshape(-1, 4).sum(axis=1)
    return 2.0 * occ - z_val


def band_energy(D, H):
    """2 Tr[D H]."""
    return 2.0 * float(np.sum(D * H))   # D, H symmetric: Tr[DH] = sum_ij D_ij H_ij


def coulomb_energy(q, n, gamma):
    """sum_i q_i V_i - 1/2 n^T gamma n, V = gamma n (charge form of Eq. Approx)."""
    V = gamma @ n
    return float(q @ V - 0.5 * n @ V)


def potential_energy(pos, n, D, m):
    """U(R; n) for the density matrix D = theta(mu0 I - H[n])."""
    h = tb.hamiltonian0(pos, m)
    q = mulliken(D, m.z_val)
    g = tb.gamma_matrix(pos, m)
    return 2.0 * float(np.sum(D * h)) + coulomb_energy(q, n, g) + tb.pair_energy(pos, m)


def forces(pos, n, D, m, q=None):
    """F_k = -dU/dR_k at constant n (see module docstring); shape (n_atoms, 3).
    q: the charges of D (default: the orthogonal Mulliken charges)."""
    nat = len(pos)
    F = np.zeros((nat, 3))
    if q is None:
        q = mulliken(D, m.z_val)
    # band term: -2 Tr[rho dh/dR_k]; each pair (i, j) appears as the block
    # h_ij and its transpose h_ji, hence the factor 4 with symmetric rho.
    ii, jj, d, r = tb.neighbour_pairs(pos, m.r_cut)
    for a, b, dv in zip(ii, jj, d):
        G = tb.sk_block_grad(dv, m)                          # d block / d(R_b - R_a)
        rho_ab = D[4 * a:4 * a + 4, 4 * b:4 * b + 4]
        g = 4.0 * np.einsum("xij,ij->x", G, rho_ab)
        F[b] -= g
        F[a] += g
    # pair term
    _, dphi = tb.pair_phi(r, m)
    for a, b, dv, rv, dp in zip(ii, jj, d, r, dphi):
        g = dp * dv / rv
        F[b] -= g
        F[a] += g
    # Coulomb term: gamma_ab = k_e / R_ab for a != b
    for a in range(nat):
        for b in range(a + 1, nat):
            dv = pos[b] - pos[a]
            rv = float(np.sqrt(dv @ dv))
            dgamma_db = -m.coulomb_k * dv / rv ** 3          # d gamma_ab / dR_b
            w = q[a] * n[b] + q[b] * n[a] - n[a] * n[b]
            F[b] -= w * dgamma_db
            F[a] += w * dgamma_db
    return F


def kinetic_energy(vel, mass, ke_unit):
    """1/2 sum_k M_k |V_k|^2 in eV (ke_unit converts amu A^2/fs^2 to eV)."""
    return 0.5 * mass * ke_unit * float(np.sum(vel * vel))
