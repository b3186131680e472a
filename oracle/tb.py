"""Oracle: orthogonal sp tight-binding model (test infrastructure only).

Follows the Appendix subsection on self-consistent-charge tight binding:
h is a Slater-Koster two-centre Hamiltonian with atomic indices i, j and
orbital labels alpha, beta (Eq. DFTB_2 with S = I); the radial dependence of
the bond integrals follows the zeta(R) form, and a fifth-order polynomial tail
t(R) on [R_1, R_cut] matches value, first and second derivative of zeta at
R_1 and sends all three to zero at R_cut (tail paragraph after the zeta(R)
equation).  gamma decays like 1/R and equals the Hubbard U on site (gamma
paragraph).  E_pair is a sum of short-range pair potentials phi(R) with the
same tail.

Readings where the paper is silent (listed in the design doc):
* zeta(R) = t0 exp(-(R - r0)/lam), i.e. A_1 = -1/lam, A_2..A_4 = 0;
* bond-integral signs ss-sigma < 0, sp-sigma > 0, pp-sigma > 0, pp-pi < 0;
* gamma_ij = k_e / R_ij for i != j (no screening), gamma_ii = U;
* phi(R) = A exp(-(R - r0p)/rho).

Pins: the Slater-Koster blocks against closed-form two-atom cases, symmetry,
rotational invariance of the spectrum, the tail conditions, and all
derivatives against central finite differences (tests/test_oracle_tb.py).
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------- radial form

def tail_coefficients(f0: float, f1: float, f2: float, r1: float, rcut: float):
    """B_0..B_5 of the cut-off tail t(R) = sum_k B_k (R - R_1)^k.

    Conditions (tail paragraph of the SCC-TB subsection): t, t', t'' equal
    the given zeta values f0, f1, f2 at R_1 and vanish at R_cut.  Solved as
    the plain 6x6 linear system of those six conditions.
    """
    d = rcut - r1
    A = np.zeros((6, 6))
    b = np.array([f0, f1, f2, 0.0, 0.0, 0.0])
    for k in range(6):
        A[0, k] = 1.0 if k == 0 else 0.0                 # t(R1)
        A[1, k] = 1.0 if k == 1 else 0.0                 # t'(R1)
        A[2, k] = 2.0 if k == 2 else 0.0                 # t''(R1)
        A[3, k] = d ** k                                 # t(Rcut)
        A[4, k] = k * d ** (k - 1) if k >= 1 else 0.0    # t'(Rcut)
        A[5, k] = k * (k - 1) * d ** (k - 2) if k >= 2 else 0.0
    return np.linalg.solve(A, b)


def _exp_radial(r, amp, r0, decay):
    """zeta(R) = amp * exp(-(R - r0)/decay) and its first two derivatives."""
    z = amp * np.exp(-(r - r0) / decay)
    return z, -z / decay, z / decay ** 2


def radial(r, amp, r0, decay, r1, rcut):
    """Radial function with optional tail: value and dR derivative.

    zeta on R < R_1, the quintic tail on [R_1, R_cut), zero beyond.  With
    R_1 == R_cut this is the literal hard cut-off.
    """
    r = np.asarray(r, dtype=np.float64)
    val = np.zeros_like(r)
    der = np.zeros_like(r)
    inner = r < r1
    z, dz, _ = _exp_radial(r[inner], amp, r0, decay)
    val[inner] = z
    der[inner] = dz
    if r1 < rcut:
        f0, f1, f2 = _exp_radial(np.float64(r1), amp, r0, decay)
        B = tail_coefficients(f0, f1, f2, r1, rcut)
        mid = (r >= r1) & (r < rcut)
        x = r[mid] - r1
        val[mid] = sum(B[k] * x ** k for k in range(6))
        der[mid] = sum(k * B[k] * x ** (k - 1) for k in range(1, 6))
    return val, der


def hopping(r, m):
    """|t(r)| and d|t|/dr of the synthetic model (model fields of synth.TBModel)."""
    return radial(r, m.t0, m.r0, m.lam, m.r_tail, m.r_cut)


def pair_phi(r, m):
    """Pair repulsion phi(R) and its derivative (E_pair term of Eq. DFTB_1)."""
    if m.pair_a == 0.0:
        z = np.zeros_like(np.asarray(r, dtype=np.float64))
        return z, z.copy()
    return radial(r, m.pair_a, m.pair_r0, m.pair_rho, m.r_tail, m.r_cut)


# ------------------------------------------------------- Slater-Koster blocks

def bond_integrals(t):
    """(V_ss_sigma, V_sp_sigma, V_pp_sigma, V_pp_pi) for hopping magnitude t."""
    return -t, t, t, -t


def sk_block(c, t):
    """4x4 block h_{i alpha, j beta} for unit vector c from atom i to atom j.

    Orbital order (s, px, py, pz).  Standard Slater-Koster two-centre table
    for s and p orbitals: E_ss = V_ss; E_s,k = c_k V_sp; E_k,s = -c_k V_sp;
    E_k,l = c_k c_l (V_pp_sigma - V_pp_pi) + delta_kl V_pp_pi.
    """
    vss, vsp, vpps, vppp = bond_integrals(t)
    B = np.empty((4, 4))
    B[0, 0] = vss
    B[0, 1:] = c * vsp
    B[1:, 0] = -c * vsp
    B[1:, 1:] = np.outer(c, c) * (vpps - vppp) + np.eye(3) * vppp
    return B


def neighbour_pairs(pos, rcut):
    """All pairs i < j closer than rcut: (i, j, d = R_j - R_i, r = |d|)."""
    n = len(pos)
    ii, jj = np.triu_indices(n, k=1)
    d = pos[jj] - pos[ii]
    r = np.sqrt(np.einsum("ij,ij->i", d, d))
    keep = r < rcut
    return ii[keep], jj[keep], d[keep], r[keep]


def hamiltonian0(pos, m):
    """Charge-independent h (N = 4 n_atoms, orbital index 4*atom + alpha).

    On-site: eps_s, eps_p on the diagonal.  Off-site: one Slater-Koster block
    per pair closer than r_cut, and its transpose in the mirrored position,
    so h is exactly symmetric.
    """
    nat = len(pos)
    N = 4 * nat
    h = np.zeros((N, N))
    onsite = np.array([m.eps_s, m.eps_p, m.eps_p, m.eps_p])
    h[np.arange(N), np.arange(N)] = np.tile(onsite, nat)
    ii, jj, d, r = neighbour_pairs(pos, m.r_cut)
    t, _ = hopping(r, m)
    for a, b, dv, rv, tv in zip(ii, jj, d, r, t):
        B = sk_block(dv / rv, tv)
        h[4 * a:4 * a + 4, 4 * b:4 * b + 4] = B
        h[4 * b:4 * b + 4, 4 * a:4 * a + 4] = B.T
    return h


def sk_block_grad(dv, m):
    """d(block)/d(d_a) for a = x, y, z, with d = R_j - R_i; shape (3, 4, 4).

    Chain rule through the direction cosines (dc_k/dd_a = (delta_ka - c_k
    c_a)/r) and the radial magnitude (dt/dd_a = t'(r) c_a).
    """
    r = float(np.sqrt(dv @ dv))
    c = dv / r
    t, dt = hopping(np.array([r]), m)
    t, dt = float(t[0]), float(dt[0])
    vss, vsp, vpps, vppp = bond_integrals(t)
    dvss, dvsp, dvpps, dvppp = bond_integrals(dt)
    G = np.zeros((3, 4, 4))
    for a in range(3):
        dc = (np.eye(3)[a] - c * c[a]) / r        # d c / d d_a
        rad = c[a]                                 # d r / d d_a
        G[a, 0, 0] = dvss * rad
        G[a, 0, 1:] = dc * vsp + c * dvsp * rad
        G[a, 1:, 0] = -(dc * vsp + c * dvsp * rad)
        G[a, 1:, 1:] = ((np.outer(dc, c) + np.outer(c, dc)) * (vpps - vppp)
                        + np.outer(c, c) * (dvpps - dvppp) * rad
                        + np.eye(3) * dvppp * rad)
    return G


# ------------------------------------------------------------------ Coulomb

def gamma_matrix(pos, m):
    """gamma_ij = k_e / R_ij (i != j), gamma_ii = U (gamma paragraph)."""
    d = pos[None, :, :] - pos[:, None, :]
    r = np.sqrt(np.sum(d * d, axis=2))
    g = np.empty_like(r)
    off = ~np.eye(len(pos), dtype=bool)
    g[off] = m.coulomb_k / r[off]
    g[~off] = m.hubbard_u
    return g


def onsite_potential(pos, n, m):
    """V_i = sum_l gamma_il n_l, the charge shift of Eq. DFTB_2 (S = I)."""
    return gamma_matrix(pos, m) @ n


def hamiltonian(pos, n, m):
    """H[n] = h + diag over the orbitals of atom i of V_i (Eq. DFTB_2, S = I)."""
    h = hamiltonian0(pos, m)
    if n is not None:
        V = onsite_potential(pos, np.asarray(n, dtype=np.float64), m)
        h[np.diag_indices_from(h)] += np.repeat(V, 4)
    return h


def pair_energy(pos, m):
    """E_pair = sum over pairs phi(R_ij)."""
    _, _, _, r = neighbour_pairs(pos, m.r_cut)
    phi, _ = pair_phi(r, m)
    return float(np.sum(phi))
