"""Pins of the charge / energy / force / XL-BOMD oracle."""
import numpy as np
import pytest

import synth
from oracle import eig, observables, tb, xlbomd

MD = synth.MD_MODEL.with_(pair_a=5.0)


def _system():
    pos = synth.lattice_positions((2, 2, 2), seed=21)
    return pos, 2 * len(pos)


def test_mulliken_sum_and_band_energy():
    pos, nocc = _system()
    n = np.linspace(-0.2, 0.2, len(pos))
    H = tb.hamiltonian(pos, n, MD)
    D, ev, _ = eig.density_matrix(H, nocc)
    q = observables.mulliken(D)
    assert abs(q.sum()) < 1e-12
    assert observables.band_energy(D, H) == pytest.approx(eig.band_energy_from_eigenvalues(ev, nocc), abs=1e-10)


def _U(pos, n, nocc):
    H = tb.hamiltonian(pos, n, MD)
    D, _, gap = eig.density_matrix(H, nocc)
    assert gap > 1e-3
    return observables.potential_energy(pos, n, D, MD), D


def test_forces_are_gradient_of_energy_at_constant_n():
    pos, nocc = _system()
    n = np.array([0.3, -0.1, 0.05, -0.2, 0.1, -0.15, 0.0, 0.0])
    U0, D = _U(pos, n, nocc)
    F = observables.forces(pos, n, D, MD)
    h = 1e-4
    for k in range(len(pos)):
        for a in range(3):
            p, m_ = pos.copy(), pos.copy()
            p[k, a] += h
            m_[k, a] -= h
            fd = -(_U(p, n, nocc)[0] - _U(m_, n, nocc)[0]) / (2 * h)
            assert F[k, a] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    np.testing.assert_allclose(F.sum(axis=0), 0.0, atol=1e-10)   # no net force


def test_energy_at_self_consistency_and_harris_foulkes_quadratic():
    pos, nocc = _system()
    m = MD
    qs, _ = xlbomd.scf(pos, m, nocc, beta=0.3, tol=1e-12, solver="jacobi")
    g = tb.gamma_matrix(pos, m)

    def U(n):
        H = tb.hamiltonian(pos, n, m)
        D, _, _ = eig.density_matrix(H, nocc)
        return observables.potential_energy(pos, n, D, m), D

    U0, D0 = U(qs)
    E_scc = 2 * np.sum(D0 * tb.hamiltonian0(pos, m)) + 0.5 * qs @ g @ qs + tb.pair_energy(pos, m)
    assert U0 == pytest.approx(E_scc, abs=1e-10)
    v = np.linspace(1, -1, len(pos))
    v -= v.mean()
    errs = [abs(U(qs + s * v)[0] - U0) for s in (1e-2, 5e-3)]
    # error of second order in (n - q*): halving s quarters the error
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)


def test_dissipation_coefficients_conserve_linear_histories():
    c = np.array(xlbomd.K5_C)
    k = np.arange(len(c))
    assert c.sum() == 0 and (k * c).sum() == 0
    hist = [np.full(3, 1.0 + 0.1 * j) for j in range(6)]      # linear in t
    assert np.allclose(xlbomd.nvt_dissipation(hist, 0.018, c), 0.0)


def test_time_reversible_without_dissipation():
    pos, nocc = _system()
    m = MD
    vel = synth.maxwell_velocities(len(pos), 300.0, m.mass, seed=5)
    qs, _ = xlbomd.scf(pos, m, nocc, beta=0.3, tol=1e-12, solver="jacobi")
    opts = xlbomd.XLOptions(alpha=0.0, solver="jacobi")
    st = xlbomd.init_state(pos, vel, m, nocc, opts, qs)
    fwd, _ = xlbomd.run(st, m, nocc, opts, 20)
    # reverse: flip velocities; the reverse history is [n_20, n_21] with n_21 the
    # next forward Verlet value, so the first reverse step reproduces n_19
    n21 = xlbomd.verlet_n(fwd.hist, fwd.q, opts.kappa, opts.alpha, opts.c)
    back = xlbomd.XLState(fwd.pos.copy(), -fwd.vel, [fwd.hist[0], n21] + fwd.hist[1:-1],
                          fwd.q, fwd.F, fwd.U)
    rev, _ = xlbomd.run(back, m, nocc, opts, 20)
    assert np.max(np.abs(rev.pos - pos)) < 1e-9
    assert np.max(np.abs(rev.vel + vel)) < 1e-9
    assert np.max(np.abs(rev.hist[0] - qs)) < 1e-9


def test_energy_error_scales_as_dt_squared():
    """Energy conservation of the integrator: the fluctuation of E_tot over a fixed
    time span shrinks ~4x when the time step is halved (second-order Verlet)."""
    m = synth.MD_MODEL
    pos, nocc = _system()
    vel = synth.maxwell_velocities(len(pos), 300.0, m.mass, seed=6)
    qs, _ = xlbomd.scf(pos, m, nocc, beta=0.3, tol=1e-12, solver="jacobi")
    dev = []
    for dt in (0.25, 0.125):
        opts = xlbomd.XLOptions(solver="jacobi", dt_fs=dt)
        st = xlbomd.init_state(pos, vel, m, nocc, opts, qs)
        e0 = xlbomd.total_energy(st, m)
        _, log = xlbomd.run(st, m, nocc, opts, int(round(25.0 / dt)))
        et = np.array([r["etot"] for r in log])
        dev.append(np.max(np.abs(et - e0)))
        assert max(r["max_q_minus_n"] for r in log) < 1e-2   # n follows q without SCF
    assert dev[0] / dev[1] == pytest.approx(4.0, rel=0.25)


def test_md_pair_amplitude_zeroes_the_virial():
    """The frozen pair amplitude of the MD model is the zero-virial one."""
    from oracle.calibrate_pair import virial_at, zero_virial_amplitude
    m = synth.MD_MODEL
    A, w0, q = zero_virial_amplitude(m)
    assert A == pytest.approx(m.pair_a, abs=1e-5)
    pos = synth.lattice_positions((4, 4, 4), jitter=0.0, seed=0)
    assert abs(virial_at(pos, q, m, 2 * len(pos), m.pair_a)) < 1e-5 * abs(w0)
    # the charge-ordered state this balances: +-4 e on the two sublattices
    assert np.allclose(np.abs(q), 4.0, atol=0.05)



def test_gapped_md_pair_amplitude_zeroes_the_virial():
    """The gapped MD model's frozen pair amplitude gives its self-consistent
    unjittered 2.0 A lattice zero virial (closed-shell atoms, 2 electrons)."""
    from oracle.calibrate_pair import virial_at, zero_virial_amplitude
    m = synth.GAPPED_MD_MODEL
    A, w0, q = zero_virial_amplitude(m, spacing=synth.GAPPED_SPACING, n0=np.zeros(64))
    assert A == pytest.approx(m.pair_a, abs=1e-5)
    pos = synth.lattice_positions((4, 4, 4), spacing=synth.GAPPED_SPACING, jitter=0.0, seed=0)
    assert abs(virial_at(pos, q, m, len(pos), m.pair_a)) < 1e-5 * abs(w0)
    assert np.abs(q).max() < 1e-2          # closed shells stay nearly neutral

def test_pair_repulsion_walls_off_ion_collapse():
    """A +-4 e pair: with rho = 0.15 A the energy rises again below ~1 A; with
    rho = 0.3 A at its own zero-virial amplitude it falls all the way in."""
    from oracle.calibrate_pair import zero_virial_amplitude
    k = synth.COULOMB_EV_A * 16.0

    def pair(m, r):
        return float(tb.pair_phi(np.array([r]), m)[0][0]) - k / r

    m = synth.MD_MODEL
    assert pair(m, 0.9) > pair(m, 1.5) and pair(m, 0.7) > pair(m, 0.9)
    soft = m.with_(pair_rho=0.3)
    soft = soft.with_(pair_a=zero_virial_amplitude(soft)[0])
    rs = np.linspace(0.2, 1.5, 27)
    e = np.array([pair(soft, r) for r in rs])
    assert np.all(np.diff(e) > 0)            # monotonic: no barrier anywhere


def test_stability_bound_of_the_charge_integration():
    """J = dq/dn by finite differences; the undamped Verlet step for n is
    stable for kappa < 4 / max eig(I - J)."""
    dims = (4, 4, 4)
    pos = synth.lattice_positions(dims, seed=21)
    m = synth.MD_MODEL
    q, _ = xlbomd.scf(pos, m, 128, beta=1.0, tol=1e-11, n0=synth.checkerboard_charges(dims))
    # no charge coupling: H does not depend on n, J = 0 and the bound is the
    # free-oscillator limit kappa < 4
    J0 = xlbomd.charge_response(pos, q, m.with_(hubbard_u=0.0, coulomb_k=0.0), 128)
    assert np.abs(J0).max() == 0.0 and xlbomd.stability_bound(J0) == 4.0
    # the scalar case reproduces the root condition of z^2 - (2 - kappa mu) z + 1
    assert xlbomd.stability_bound(np.array([[-1.0]])) == pytest.approx(2.0)
    assert xlbomd.stability_bound(np.array([[1.5]])) == 0.0
    # the charge-ordered state: a small response, kappa = 0.91 well inside
    bound = xlbomd.check_stability(pos, q, m, 128, 0.91)
    assert 3.5 < bound <= 4.0
    # a large on-site U (metallic charge response) leaves almost no room
    with pytest.raises(ValueError):
        xlbomd.check_stability(pos, np.zeros(64), m.with_(hubbard_u=40.0), 128, 0.91)
    opts = xlbomd.XLOptions(check_stability=True)
    with pytest.raises(ValueError):
        xlbomd.init_state(pos, np.zeros((64, 3)), m.with_(hubbard_u=40.0), 128, opts, np.zeros(64))


def test_mulliken_charges_of_a_diagonal_projector():
    """Atom-major orbitals (s, px, py, pz of atom 0, then atom 1, ...): charges of
    a diagonal D worked by hand, q_i = 2 (sum of atom i's occupations) - 4."""
    D = np.diag([1, 1, 0, 0,  1, 1, 1, 1,  0, 0, 0.5, 0.5,  0.25, 0, 0, 0.75]).astype(float)
    np.testing.assert_array_equal(observables.mulliken(D), [0.0, 4.0, -2.0, -2.0])


def test_auxiliary_charge_verlet_closed_form():
    """With q held fixed and no dissipation, Eq. Verl_n reads
    e_{t+1} = (2 - kappa) e_t - e_{t-1} for e = n - q, solved exactly by
    e_t = cos(theta t) with cos(theta) = 1 - kappa / 2 when e_0 = 1 and
    e_{-1} = cos(theta).  A wrong sign of the kappa term grows instead."""
    kappa = 0.91
    theta = np.arccos(1.0 - kappa / 2.0)
    q = np.array([0.3, -0.7])
    hist = [q + 1.0, q + np.cos(theta)] + [q] * 4
    c = np.array(xlbomd.K5_C)
    for t in range(1, 60):
        n_next = xlbomd.verlet_n(hist, q, kappa, 0.0, c)
        hist = [n_next] + hist[:-1]
        np.testing.assert_allclose(hist[0] - q, np.cos(theta * t), atol=1e-12)


def test_dissipation_applies_c_k_to_n_t_minus_k():
    """The K = 5 coefficients on histories n_{t-k dt} = k^2 and k^3, worked by
    hand: sum_k c_k k^2 = -6 and sum_k c_k k^3 = 0; with the coefficients
    applied in reverse order the cubic history would give -90."""
    c = np.array(xlbomd.K5_C)
    alpha = 0.018
    quad = [np.full(2, float(k * k)) for k in range(6)]
    cube = [np.full(2, float(k ** 3)) for k in range(6)]
    np.testing.assert_allclose(xlbomd.nvt_dissipation(quad, alpha, c), -6.0 * alpha, atol=1e-15)
    np.testing.assert_allclose(xlbomd.nvt_dissipation(cube, alpha, c), 0.0, atol=1e-13)


def _step_matrix(kappa, alpha, c):
    """The linear map (e_t, ..., e_{t-5}) -> (e_{t+1}, ..., e_{t-4}) of the
    deviation e = n - q under the oracle's Eq. Verl_n step with q held fixed,
    built by applying the step to unit histories."""
    K1 = len(c)
    M = np.zeros((K1, K1))
    q = np.zeros(1)
    for j in range(K1):
        hist = [np.array([1.0 if i == j else 0.0]) for i in range(K1)]
        M[0, j] = xlbomd.verlet_n(hist, q, kappa, alpha, c)[0]
    M[1:, :-1] = np.eye(K1 - 1)
    return M


def test_dissipation_damps_the_auxiliary_charges():
    """At a fixed q the K = 5 set damps every mode of n - q strictly (spectral
    radius 0.986 at the integrator's kappa = 0.91, 0.913 at 1.82); without
    dissipation the two Verlet modes stay on the unit circle (reversible);
    with the coefficients in reverse order or of the opposite sign the
    recurrence grows."""
    c = np.array(xlbomd.K5_C)
    rho = lambda kap, a, cc: float(np.abs(np.linalg.eigvals(_step_matrix(kap, a, cc))).max())
    for kap, expect in ((0.5 * xlbomd.K5_KAPPA, 0.98565), (xlbomd.K5_KAPPA, 0.91251)):
        assert rho(kap, xlbomd.K5_ALPHA, c) == pytest.approx(expect, abs=1e-5)
        assert rho(kap, 0.0, c) == pytest.approx(1.0, abs=1e-7)
        assert rho(kap, xlbomd.K5_ALPHA, c[::-1]) > 1.02
        assert rho(kap, xlbomd.K5_ALPHA, -c) > 1.02
