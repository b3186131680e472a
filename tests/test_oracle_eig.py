"""Pins of the Jacobi + aufbau oracle against closed forms and a library eigensolver."""
import numpy as np
import pytest

import synth
from oracle import eig, tb


def test_diagonal_matrix_closed_form():
    d = np.array([3.0, -1.0, 2.0, -5.0, 0.5])
    w, V = eig.jacobi_eigh(np.diag(d))
    np.testing.assert_array_equal(w, np.sort(d))
    # eigenvectors are unit coordinate vectors
    np.testing.assert_allclose(np.abs(V).sum(axis=0), 1.0, atol=0)
    rho, _, gap = eig.density_matrix(np.diag(d), 2)
    expect = np.diag((d <= -1.0).astype(float))      # two lowest: -5, -1
    np.testing.assert_array_equal(rho, expect)
    assert gap == pytest.approx(0.5 - (-1.0))


@pytest.mark.parametrize("a,b,c", [(1.0, 0.3, -2.0), (-4.0, 2.0, -4.0), (0.0, -1e-3, 5.0)])
def test_two_by_two_closed_form(a, b, c):
    A = np.array([[a, b], [b, c]])
    mean, half = 0.5 * (a + c), np.hypot(0.5 * (a - c), b)
    w, V = eig.jacobi_eigh(A)
    np.testing.assert_allclose(w, [mean - half, mean + half], rtol=0, atol=1e-14)
    # lower eigenvector satisfies (A - w0) v = 0
    np.testing.assert_allclose(A @ V[:, 0], w[0] * V[:, 0], atol=1e-14)
    rho, _, _ = eig.density_matrix(A, 1)
    np.testing.assert_allclose(rho, np.outer(V[:, 0], V[:, 0]), atol=1e-15)


def test_matches_library_eigensolver_random():
    rng = np.random.default_rng(7)
    M = rng.normal(size=(60, 60))
    A = M + M.T
    w, V = eig.jacobi_eigh(A)
    wl = np.linalg.eigh(A)[0]
    np.testing.assert_allclose(w, wl, atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(60), atol=1e-13)
    np.testing.assert_allclose(V @ np.diag(w) @ V.T, A, atol=1e-12)


def test_tb_projector_properties_and_library():
    w = synth.small_workload((3, 2, 2), 11)
    H = tb.hamiltonian(w.positions(), None, synth.STATIC_MODEL)
    rho, ev, gap = eig.density_matrix(H, w.n_occ)
    wl, Vl = np.linalg.eigh(H)
    np.testing.assert_allclose(ev, wl, atol=1e-12)
    assert gap > 1e-6
    ref = Vl[:, :w.n_occ] @ Vl[:, :w.n_occ].T
    np.testing.assert_allclose(rho, ref, atol=1e-12)
    assert np.linalg.norm(rho @ rho - rho) < 1e-12
    assert abs(np.trace(rho) - w.n_occ) < 1e-12
    assert np.linalg.norm(H @ rho - rho @ H) < 1e-11
    assert eig.band_energy_from_eigenvalues(ev, w.n_occ) == pytest.approx(
        2.0 * np.sum(rho * H), abs=1e-10)
