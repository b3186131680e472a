"""Pins of the finite-temperature oracle: the definition against brute force and
limits, the recursion against the definition within its error bound."""
import numpy as np
import pytest

import synth
from oracle import eig, fermi, tb


@pytest.fixture(scope="module")
def system():
    w = synth.small_workload((3, 3, 3), 4)
    return w, tb.hamiltonian(w.positions(), None, synth.STATIC_MODEL)


def test_fermi_definition_brute_force(system):
    w, H = system
    D, mu, f = fermi.fermi_density(H, w.n_occ, 0.5)
    assert f.sum() == pytest.approx(w.n_occ, abs=1e-9)
    assert np.trace(D) == pytest.approx(w.n_occ, abs=1e-9)
    e, V = np.linalg.eigh(H)
    for i in range(0, len(e), 17):                       # spot-check f(e_i) = 1/(1 + exp(beta (e_i - mu)))
        assert f[i] == pytest.approx(1.0 / (1.0 + np.exp((e[i] - mu) / 0.5)), rel=1e-12)
    np.testing.assert_allclose(D @ V, V * f, atol=1e-10)  # eigenvectors shared, eigenvalues f


def test_fermi_zero_temperature_limit():
    """A gapped system: as kT -> 0 the Fermi operator becomes the projector."""
    w = synth.gapped_workload(2)
    H = tb.hamiltonian0(w.positions(), synth.GAPPED_MODEL)
    P, _, gap = eig.density_matrix(H, w.n_occ)
    assert gap > 4.0
    D, _, _ = fermi.fermi_density(H, w.n_occ, 0.05)
    assert np.abs(D - P).max() < 1e-12


def test_recursion_matches_definition_within_its_bound(system):
    w, H = system
    kT = 0.5
    D, mu, f = fermi.fermi_density(H, w.n_occ, kT)
    e = np.linalg.eigvalsh(H)
    errs = []
    for n in (8, 10, 12, 14):
        X = fermi.recursive_fermi(H, mu, kT, n)
        err = np.abs(X - D).max()
        # exponent error (beta |e - mu| / 2^n)^2 / 12 times the slope f (1 - f) beta |e - mu|
        x = np.abs(e - mu) / kT
        bound = np.max(f * (1 - f) * x * (x / 2.0 ** n) ** 2 / 12.0) * len(e)
        assert err <= bound + 1e-12
        errs.append(err)
    # the error falls as 2^(-2n): 16x per two steps, down to the rounding floor
    for a, b in zip(errs, errs[1:]):
        assert 12.0 < a / b < 20.0
    assert np.abs(fermi.recursive_fermi(H, mu, kT, 18) - D).max() < 1e-10


def test_canonical_recursion(system):
    w, H = system
    X, mu_x, its = fermi.recursive_fermi_canonical(H, w.n_occ, 0.5, 18)
    D, mu, _ = fermi.fermi_density(H, w.n_occ, 0.5)
    assert np.trace(X) == pytest.approx(w.n_occ, abs=1e-9)
    assert mu_x == pytest.approx(mu, abs=1e-7)
    assert np.abs(X - D).max() < 1e-8
    assert its < 20


def test_entropy_limits():
    assert fermi.entropy([0.0, 1.0, 1.0, 0.0]) == 0.0
    assert fermi.entropy(np.full(6, 0.5)) == pytest.approx(2 * 6 * np.log(2.0), rel=1e-15)
    # symmetric under f -> 1 - f, and positive
    f = np.array([0.1, 0.3, 0.8, 0.999])
    assert fermi.entropy(f) == pytest.approx(fermi.entropy(1.0 - f), rel=1e-14)
    assert fermi.entropy(f) > 0.0


def test_finite_temperature_forces_are_gradient_of_free_energy():
    """At T_e > 0 the constant-n force expression with the Fermi D is -dA/dR,
    A = U - T_e S, mu re-solved at every geometry (central differences)."""
    from oracle import observables
    m = synth.MD_MODEL.with_(pair_a=5.0)
    pos = synth.lattice_positions((2, 2, 2), seed=21)
    n_occ = 2 * len(pos)
    n = np.array([0.3, -0.1, 0.05, -0.2, 0.1, -0.15, 0.0, 0.0])
    kT = 0.5
    _, D, _ = fermi.free_energy(pos, n, m, n_occ, kT)
    F = observables.forces(pos, n, D, m)
    h = 1e-4
    for k in range(len(pos)):
        for a in range(3):
            p, q = pos.copy(), pos.copy()
            p[k, a] += h
            q[k, a] -= h
            fd = -(fermi.free_energy(p, n, m, n_occ, kT)[0] - fermi.free_energy(q, n, m, n_occ, kT)[0]) / (2 * h)
            assert F[k, a] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    # without the entropy term the same differences miss the force
    def U(pp):
        return observables.potential_energy(pp, n, fermi.free_energy(pp, n, m, n_occ, kT)[1], m)
    p, q = pos.copy(), pos.copy()
    p[0, 0] += h
    q[0, 0] -= h
    assert abs(-(U(p) - U(q)) / (2 * h) - F[0, 0]) > 1e-4


def test_xlbomd_evaluate_at_finite_temperature_is_the_free_energy():
    """The integrator's evaluation at kT > 0 returns the Fermi D, its charges,
    U - T_e S and the forces of that D (the pinned free-energy gradient)."""
    from oracle import observables, xlbomd
    m = synth.MD_MODEL.with_(pair_a=5.0)
    pos = synth.lattice_positions((2, 2, 2), seed=21)
    n = np.linspace(-0.1, 0.1, len(pos))
    ev = xlbomd.evaluate(pos, n, m, 2 * len(pos), kT=1.5)
    A, D, mu = fermi.free_energy(pos, n, m, 2 * len(pos), 1.5)
    assert ev["U"] == pytest.approx(A, rel=1e-14)
    np.testing.assert_allclose(ev["D"], D, atol=1e-14)
    np.testing.assert_allclose(ev["q"], observables.mulliken(D, m.z_val), atol=1e-14)
    np.testing.assert_allclose(ev["F"], observables.forces(pos, n, D, m), atol=1e-12)
    assert abs(np.trace(D) - 2 * len(pos)) < 1e-10
    # with an overlap the evaluation is the non-orthogonal free energy (pinned
    # in test_oracle_nonorth.py); its Fermi operator keeps Tr[D S] = n_occ
    from oracle import nonorth
    mo = m.with_(overlap_s0=0.05)
    evo = xlbomd.evaluate(pos, n, mo, 2 * len(pos), kT=1.5)
    assert abs(np.trace(evo["D"] @ nonorth.overlap(pos, mo)) - 2 * len(pos)) < 1e-9
