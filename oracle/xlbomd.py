"""Oracle: optimisation-free XL-BOMD for the orthogonal T_e = 0 model.

Test infrastructure only.

* Initialisation (General remarks subsection): converge the charges
  self-consistently, then set n = q for the whole history.  The SCF here is
  plain linear mixing n <- n + beta (q[n] - n) until max|q - n| < tol.
* Auxiliary charges (Eq. Verl_n with sigma -> q, Eq. EL_Orth_b):
  n_{t+dt} = 2 n_t - n_{t-dt} + kappa (q_t - n_t) + alpha sum_{k=0}^{K} c_k n_{t-k dt}.
  kappa, alpha, c_k with K = 5 come from the cited dissipation paper, which the
  text does not reprint; kappa is rescaled by 1/2 (General remarks).  Reading:
  kappa = 1.82 / 2, alpha = 0.018, c = (-6, 14, -8, -3, 4, -1); they are
  inputs, and what the tests pin is sum c_k = 0 and sum k c_k = 0 (the
  dissipation vanishes on histories linear in t), time reversibility for
  alpha = 0, and that at a fixed q the set damps every mode of n - q while
  reversed or negated coefficients make the recurrence grow.
* Nuclei: velocity Verlet with the forces of ``observables.forces`` at the
  new (R, n) — one density-matrix construction per step.
* Constant of motion: E_tot = kinetic + U(R; n) (Eq. EtotOrth, S = 0).

The density matrix comes from the oracle SP2 (or Jacobi when requested).
A model with a nonzero overlap (overlap_s0 > 0) takes the non-orthogonal
H[n], density matrix, charges, energy and forces of the nonorth module (its
readings); the integrators are unchanged.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import synth

from . import eig, fermi, nonorth, observables, sp2, tb

K5_KAPPA = 1.82
K5_ALPHA = 0.018
K5_C = (-6.0, 14.0, -8.0, -3.0, 4.0, -1.0)


@dataclasses.dataclass
class XLOptions:
    dt_fs: float = 0.25
    kappa: float = 0.5 * K5_KAPPA
    alpha: float = K5_ALPHA
    c: tuple = K5_C
    solver: str = "sp2"           # "sp2" or "jacobi"
    sp2_tol: float = 1e-10
    check_stability: bool = False  # refuse kappa outside the stability bound at t = 0
    kT: float = 0.0               # > 0: finite electronic temperature (eV)


def density(H, n_occ, solver="sp2", tol=1e-10):
    if solver == "jacobi":
        D, _, _ = eig.density_matrix(H, n_occ)
        return D
    r = sp2.sp2(H, n_occ, tol=tol)
    if r.status not in ("converged", "stalled"):
        raise RuntimeError(f"oracle SP2 ended with status {r.status}")
    return r.D


def _nonorth(m):
    return getattr(m, "overlap_s0", 0.0) > 0.0


def nonorth_density(H, S, n_occ, solver="sp2", tol=1e-10):
    """rho of the generalized eigenproblem H c = e S c (Eq. DM_perp with the
    Loewdin factor): solver "jacobi" takes the projector of Z H Z by Jacobi,
    "sp2" by the oracle SP2; Z from Jacobi eigenpairs of S in both."""
    if solver == "jacobi":
        Z = nonorth.loewdin_factor(S)
        Hp = Z @ H @ Z
        Dp, _, _ = eig.density_matrix(0.5 * (Hp + Hp.T), n_occ)
        return Z @ Dp @ Z
    rho, _, _, r = nonorth.density_matrix(H, S, n_occ, tol=tol)
    if r.status not in ("converged", "stalled"):
        raise RuntimeError(f"oracle SP2 ended with status {r.status}")
    return rho


def charges(pos, n, m, n_occ, solver="sp2"):
    """Charges of the density matrix of H[n] (either basis)."""
    if _nonorth(m):
        S = nonorth.overlap(pos, m)
        return nonorth.mulliken(nonorth_density(nonorth.hamiltonian(pos, n, m, S), S, n_occ, solver), S, m.z_val)
    return observables.mulliken(density(tb.hamiltonian(pos, n, m), n_occ, solver), m.z_val)


def evaluate(pos, n, m, n_occ, solver="sp2", tol=1e-10, want_forces=True, kT=0.0):
    """One density-matrix construction at (R, n): returns dict of q, U, F, D.
    kT > 0: D is the Fermi operator (definition; in a non-orthogonal basis
    that of the generalized eigenproblem) and U the free energy U - T_e S
    (Eq. Entropy), whose constant-n gradient the forces of D are."""
    if kT > 0.0:
        if _nonorth(m):
            S = nonorth.overlap(pos, m)
            H = nonorth.hamiltonian(pos, n, m, S)
            D, W, mu, f = nonorth.fermi_density_matrix(H, S, n_occ, kT)
            q = nonorth.mulliken(D, S, m.z_val)
            U = nonorth.potential_energy(pos, n, D, m, S) - kT * fermi.entropy(f)
            F = nonorth.forces(pos, n, D, m, S, W) if want_forces else None
            return {"q": q, "U": U, "F": F, "D": D, "H": H, "S": S, "W": W, "mu": mu}
        H = tb.hamiltonian(pos, n, m)
        D, mu, f = fermi.fermi_density(H, n_occ, kT)
        q = observables.mulliken(D, m.z_val)
        U = observables.potential_energy(pos, n, D, m) - kT * fermi.entropy(f)
        F = observables.forces(pos, n, D, m) if want_forces else None
        return {"q": q, "U": U, "F": F, "D": D, "H": H, "mu": mu}
    if _nonorth(m):
        S = nonorth.overlap(pos, m)
        H = nonorth.hamiltonian(pos, n, m, S)
        D = nonorth_density(H, S, n_occ, solver, tol)
        q = nonorth.mulliken(D, S, m.z_val)
        U = nonorth.potential_energy(pos, n, D, m, S)
        F = nonorth.forces(pos, n, D, m, S) if want_forces else None
        return {"q": q, "U": U, "F": F, "D": D, "H": H, "S": S}
    H = tb.hamiltonian(pos, n, m)
    D = density(H, n_occ, solver, tol)
    q = observables.mulliken(D, m.z_val)
    U = observables.potential_energy(pos, n, D, m)
    F = observables.forces(pos, n, D, m) if want_forces else None
    return {"q": q, "U": U, "F": F, "D": D, "H": H}


def scf(pos, m, n_occ, beta=0.02, tol=1e-10, max_iter=20000, n0=None,
        solver="sp2"):
    """Self-consistent charges by linear mixing; returns (q*, iterations)."""
    n = np.zeros(len(pos)) if n0 is None else np.array(n0, dtype=np.float64)
    for it in range(max_iter):
        q = charges(pos, n, m, n_occ, solver)
        if np.max(np.abs(q - n)) < tol:
            return q, it + 1
        n = n + beta * (q - n)
    raise RuntimeError("oracle SCF did not converge")


def nvt_dissipation(hist, alpha, c):
    """alpha * sum_k c_k n_{t - k dt}; hist[0] = n_t, hist[k] = n_{t-k dt}."""
    return alpha * sum(ck * hk for ck, hk in zip(c, hist))


def verlet_n(hist, q, kappa, alpha, c):
    """Eq. Verl_n: the next auxiliary charges from the history and q_t."""
    n_t, n_tm1 = hist[0], hist[1]
    return 2.0 * n_t - n_tm1 + kappa * (q - n_t) + nvt_dissipation(hist, alpha, c)


@dataclasses.dataclass
class XLState:
    pos: np.ndarray
    vel: np.ndarray
    hist: list               # [n_t, n_{t-dt}, ..., n_{t-K dt}]
    q: np.ndarray
    F: np.ndarray
    U: float
    step: int = 0


def charge_response(pos, n, m, n_occ, h=1e-5, solver="sp2"):
    """J = dq/dn at (R, n): the Mulliken charges of theta(mu0 I - H[n]) by
    central differences in each n_k (2 n_atoms density matrices)."""
    nat = len(pos)
    J = np.zeros((nat, nat))
    for k in range(nat):
        e = np.zeros(nat)
        e[k] = h
        qp = observables.mulliken(density(tb.hamiltonian(pos, n + e, m), n_occ, solver), m.z_val)
        qm = observables.mulliken(density(tb.hamiltonian(pos, n - e, m), n_occ, solver), m.z_val)
        J[:, k] = (qp - qm) / (2.0 * h)
    return J


def stability_bound(J):
    """Largest kappa for which the undamped auxiliary-charge step
    n_{t+1} = 2 n_t - n_{t-1} + kappa (q[n_t] - n_t) is stable about a fixed
    point (Eq. Verl_n without dissipation, linearised): along an eigenvector
    of I - J with eigenvalue mu the step is z^2 - (2 - kappa mu) z + 1 = 0,
    whose roots stay on the unit circle iff 0 <= kappa mu <= 4.  Returns
    4 / max mu (0 if some mu < 0: no kappa is stable)."""
    mu = np.linalg.eigvals(np.eye(len(J)) - J).real
    if mu.min() < 0.0:
        return 0.0
    return 4.0 / mu.max()


def check_stability(pos, n, m, n_occ, kappa, solver="sp2"):
    """Raise ValueError when kappa is not below the stability bound at (R, n)."""
    bound = stability_bound(charge_response(pos, n, m, n_occ, solver=solver))
    if not kappa < bound:
        raise ValueError(f"kappa = {kappa} is outside the stability bound {bound:.4g} of the "
                         "auxiliary-charge integration")
    return bound


def init_state(pos, vel, m, n_occ, opts: XLOptions, n0):
    """State at t = 0 with n_{-k dt} = n0 for all k (n0 = SCF charges)."""
    n0 = np.array(n0, dtype=np.float64)
    if opts.check_stability:
        check_stability(pos, n0, m, n_occ, opts.kappa, opts.solver)
    ev = evaluate(pos, n0, m, n_occ, opts.solver, opts.sp2_tol, kT=opts.kT)
    hist = [n0.copy() for _ in range(len(opts.c))]
    return XLState(pos.copy(), vel.copy(), hist, ev["q"], ev["F"], ev["U"])


def total_energy(st: XLState, m):
    return observables.kinetic_energy(st.vel, m.mass, synth.KE_EV) + st.U


def step(st: XLState, m, n_occ, opts: XLOptions) -> XLState:
    """One XL-BOMD step: half kick, drift, n update, new D, forces, half kick."""
    dt = opts.dt_fs
    acc = synth.ACC_A_FS2 / m.mass
    v_half = st.vel + 0.5 * dt * acc * st.F
    pos = st.pos + dt * v_half
    n_new = verlet_n(st.hist, st.q, opts.kappa, opts.alpha, opts.c)
    ev = evaluate(pos, n_new, m, n_occ, opts.solver, opts.sp2_tol, kT=opts.kT)
    vel = v_half + 0.5 * dt * acc * ev["F"]
    hist = [n_new] + st.hist[:-1]
    return XLState(pos, vel, hist, ev["q"], ev["F"], ev["U"], st.step + 1)


def run(st: XLState, m, n_occ, opts: XLOptions, n_steps: int):
    """Integrate n_steps; returns (final state, list of per-step records)."""
    log = []
    for _ in range(n_steps):
        st = step(st, m, n_occ, opts)
        log.append({"step": st.step,
                    "etot": total_energy(st, m),
                    "U": st.U,
                    "max_q_minus_n": float(np.max(np.abs(st.q - st.hist[0])))})
    return st, log
