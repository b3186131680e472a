"""Pins of the non-orthogonal oracle against the generalized eigenproblem and its invariants."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import nonorth, sp2, tb


@pytest.fixture(scope="module")
def system():
    w = synth.small_workload((3, 3, 3), 4)          # 27 atoms, N = 108
    pos = w.positions()
    m = synth.NONORTH_MODEL
    H = tb.hamiltonian(pos, None, m)
    S = nonorth.overlap(pos, m)
    return w, pos, m, H, S


def test_overlap_is_symmetric_positive_definite(system):
    _, _, _, _, S = system
    assert np.array_equal(S, S.T)
    assert np.allclose(np.diag(S), 1.0)
    assert np.linalg.eigvalsh(S).min() > 0.3
    assert np.abs(S - np.eye(len(S))).max() > 0.01      # not the identity


def test_loewdin_factor_is_a_congruence_factor(system):
    _, _, _, _, S = system
    Z = nonorth.loewdin_factor(S)
    assert np.allclose(Z.T @ S @ Z, np.eye(len(S)), atol=1e-12)
    assert np.allclose(Z, Z.T, atol=1e-14)


def test_density_matrix_equals_generalized_eigenproblem(system):
    """Definition: rho = C_occ C_occ^T with H C = S C E, C^T S C = I."""
    w, _, _, H, S = system
    rho, rho_p, Z, r = nonorth.density_matrix(H, S, w.n_occ)
    E, C = scipy.linalg.eigh(H, S)
    assert E[w.n_occ] - E[w.n_occ - 1] > 1e-4
    ref = C[:, :w.n_occ] @ C[:, :w.n_occ].T
    assert r.status == "converged"
    np.testing.assert_allclose(rho, ref, atol=1e-9)
    # invariants: idempotent in the S metric, S-trace = n_occ, neutral charges sum to 0
    np.testing.assert_allclose(rho @ S @ rho, rho, atol=1e-9)
    assert np.trace(rho @ S) == pytest.approx(w.n_occ, abs=1e-9)
    assert nonorth.mulliken(rho, S).sum() == pytest.approx(0.0, abs=1e-9)


def test_orthogonal_limit_is_the_orthogonal_path(system):
    w, pos, m, H, _ = system
    S0 = nonorth.overlap(pos, m.with_(overlap_s0=0.0))
    assert np.array_equal(S0, np.eye(len(S0)))
    rho, _, _, _ = nonorth.density_matrix(H, S0, w.n_occ)
    assert np.array_equal(rho, sp2.sp2(H, w.n_occ).D)


def test_mulliken_brute_force(system):
    w, _, _, H, S = system
    rng = np.random.default_rng(2)
    A = rng.standard_normal(S.shape)
    rho = A + A.T
    q = nonorth.mulliken(rho, S, z_val=4)
    for i in range(w.n_atoms):
        pop = sum(rho[a, b] * S[b, a] for a in range(4 * i, 4 * i + 4) for b in range(len(S)))
        assert q[i] == pytest.approx(2.0 * pop - 4.0, abs=1e-10)


def _md_system():
    m = synth.NONORTH_MODEL.with_(r_tail=3.5, pair_a=5.605396, pair_rho=0.15, overlap_s0=0.08)
    pos = synth.lattice_positions((2, 2, 2), seed=21)
    n = np.linspace(-0.3, 0.25, len(pos))
    return m, pos, n, 2 * len(pos)


def _rho(pos, n, m, nocc):
    E, C = scipy.linalg.eigh(nonorth.hamiltonian(pos, n, m), nonorth.overlap(pos, m))
    return C[:, :nocc] @ C[:, :nocc].T


def test_nonorth_forces_are_gradient_of_energy():
    """Central finite differences of U(R; n), rho the exact generalized
    projector at each displaced geometry; and the overlap term is needed."""
    from oracle import observables
    m, pos, n, nocc = _md_system()
    rho = _rho(pos, n, m, nocc)
    F = nonorth.forces(pos, n, rho, m)
    q = nonorth.mulliken(rho, nonorth.overlap(pos, m), m.z_val)
    F_no_overlap_term = observables.forces(pos, n, rho, m, q=q)
    h = 1e-5
    fd = np.zeros_like(F)
    for k in range(len(pos)):
        for a in range(3):
            pp = pos.copy()
            pp[k, a] += h
            pm = pos.copy()
            pm[k, a] -= h
            fd[k, a] = -(nonorth.potential_energy(pp, n, _rho(pp, n, m, nocc), m)
                         - nonorth.potential_energy(pm, n, _rho(pm, n, m, nocc), m)) / (2 * h)
    assert np.abs(F - fd).max() < 1e-5
    assert np.abs(F_no_overlap_term - fd).max() > 1e-2


def test_nonorth_energy_and_forces_reduce_to_orthogonal():
    from oracle import observables
    m, pos, n, nocc = _md_system()
    m0 = m.with_(overlap_s0=0.0)
    rho = _rho(pos, n, m0, nocc)
    assert np.array_equal(nonorth.hamiltonian(pos, n, m0), tb.hamiltonian(pos, n, m0))
    assert nonorth.potential_energy(pos, n, rho, m0) == observables.potential_energy(pos, n, rho, m0)
    np.testing.assert_allclose(nonorth.forces(pos, n, rho, m0), observables.forces(pos, n, rho, m0), atol=1e-12)


def test_nonorth_finite_temperature_forces_are_free_energy_gradient():
    """Finite electronic temperature in the non-orthogonal basis: central
    finite differences of the free energy U - kT S (rho and the canonical mu
    recomputed at each displaced geometry) give the forces with the
    energy-weighted W = Z f(H_perp) H_perp Z^T; the T_e = 0 form rho H rho
    in its place does not."""
    m, pos, n, nocc = _md_system()
    kT = 0.3
    A, rho, W, mu = nonorth.free_energy(pos, n, m, nocc, kT)
    S = nonorth.overlap(pos, m)
    F = nonorth.forces(pos, n, rho, m, S, W)
    F_idempotent_form = nonorth.forces(pos, n, rho, m, S)
    h = 1e-5
    fd = np.zeros_like(F)
    for k in range(len(pos)):
        for a in range(3):
            pp = pos.copy()
            pp[k, a] += h
            pm = pos.copy()
            pm[k, a] -= h
            fd[k, a] = -(nonorth.free_energy(pp, n, m, nocc, kT)[0] - nonorth.free_energy(pm, n, m, nocc, kT)[0]) / (2 * h)
    assert np.abs(F - fd).max() < 1e-5
    assert np.abs(F_idempotent_form - fd).max() > 1e-3


def test_nonorth_fermi_operator_invariants():
    """Tr[rho S] = n_occ at the canonical mu; rho = f of the generalized
    eigenproblem (scipy's generalized eigensolver, not the Loewdin route);
    with S = I it is the orthogonal Fermi operator and W = rho H; as kT -> 0
    it tends to the generalized projector."""
    from oracle import fermi
    m, pos, n, nocc = _md_system()
    S = nonorth.overlap(pos, m)
    H = nonorth.hamiltonian(pos, n, m, S)
    kT = 0.3
    rho, W, mu, f = nonorth.fermi_density_matrix(H, S, nocc, kT)
    assert np.trace(rho @ S) == pytest.approx(nocc, abs=1e-9)
    E, C = scipy.linalg.eigh(H, S)
    fg = 1.0 / (1.0 + np.exp((E - mu) / kT))
    np.testing.assert_allclose(rho, (C * fg) @ C.T, atol=1e-10)
    np.testing.assert_allclose(W, (C * (fg * E)) @ C.T, atol=1e-9)
    H0 = tb.hamiltonian(pos, n, m.with_(overlap_s0=0.0))
    rho0, W0, mu0, _ = nonorth.fermi_density_matrix(H0, np.eye(len(H0)), nocc, kT)
    D, mu_o, _ = fermi.fermi_density(H0, nocc, kT)
    np.testing.assert_allclose(rho0, D, atol=1e-10)
    assert mu0 == pytest.approx(mu_o, abs=1e-9)
    np.testing.assert_allclose(W0, rho0 @ H0, atol=1e-9)
    rho_cold, _, _, _ = nonorth.fermi_density_matrix(H, S, nocc, 1e-3)
    np.testing.assert_allclose(rho_cold, _rho(pos, n, m, nocc), atol=1e-6)


def test_xlbomd_evaluation_at_finite_temperature_in_the_nonorthogonal_basis():
    """The integrator's evaluation at kT > 0 with an overlap is the
    non-orthogonal free energy, its Fermi operator's charges and forces."""
    from oracle import xlbomd
    m, pos, n, nocc = _md_system()
    ev = xlbomd.evaluate(pos, n, m, nocc, kT=0.3)
    A, rho, W, mu = nonorth.free_energy(pos, n, m, nocc, 0.3)
    assert ev["U"] == pytest.approx(A, abs=1e-12)
    np.testing.assert_allclose(ev["D"], rho, atol=1e-14)
    np.testing.assert_allclose(ev["q"], nonorth.mulliken(rho, nonorth.overlap(pos, m), m.z_val), atol=1e-12)
    np.testing.assert_allclose(ev["F"], nonorth.forces(pos, n, rho, m, None, W), atol=1e-12)
