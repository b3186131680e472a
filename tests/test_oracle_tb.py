"""Pins of the tight-binding oracle: Slater-Koster closed forms, tail, symmetry, derivatives."""
import numpy as np
import pytest

import synth
from oracle import tb

M = synth.STATIC_MODEL
MD = synth.MD_MODEL.with_(pair_a=5.0)


def test_two_atoms_along_x_closed_form():
    # atom 1 at +x: only s-s, s-px, px-s, px-px (sigma) and py-py, pz-pz (pi)
    pos = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    h = tb.hamiltonian0(pos, M)
    t = 2.0 * np.exp(-(2.0 - 1.5) / 0.5)
    B = h[0:4, 4:8]
    expect = np.array([[-t, t, 0, 0],
                       [-t, t, 0, 0],
                       [0, 0, -t, 0],
                       [0, 0, 0, -t]])
    np.testing.assert_allclose(B, expect, atol=1e-15)
    np.testing.assert_array_equal(np.diag(h), [-8, -4, -4, -4] * 2)
    # beyond the cut-off there is no coupling
    far = tb.hamiltonian0(np.array([[0, 0, 0], [4.01, 0, 0]], float), M)
    assert not far[0:4, 4:8].any()


def test_two_atoms_along_diagonal_closed_form():
    c = np.ones(3) / np.sqrt(3.0)
    pos = np.array([[0.0, 0.0, 0.0], 1.7 * c])
    B = tb.hamiltonian0(pos, M)[0:4, 4:8]
    t = 2.0 * np.exp(-(1.7 - 1.5) / 0.5)
    # pp block: c_k c_l (V_pps - V_ppp) + delta_kl V_ppp = (2t/3) + delta(-t)
    np.testing.assert_allclose(B[1:, 1:], np.full((3, 3), 2 * t / 3) - t * np.eye(3), atol=1e-14)
    np.testing.assert_allclose(B[0, 1:], t * c, atol=1e-14)
    np.testing.assert_allclose(B[1:, 0], -t * c, atol=1e-14)


def test_hamiltonian_symmetric_and_rotation_invariant():
    pos = synth.lattice_positions((3, 3, 2), seed=4)
    h = tb.hamiltonian0(pos, M)
    assert np.array_equal(h, h.T)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    h2 = tb.hamiltonian0(pos @ R.T + 3.0, M)
    np.testing.assert_allclose(np.linalg.eigvalsh(h), np.linalg.eigvalsh(h2), atol=1e-12)


def test_tail_matches_and_vanishes():
    r1, rc = MD.r_tail, MD.r_cut
    eps = 1e-7
    v_in, d_in = tb.hopping(np.array([r1 - eps]), MD)
    v_out, d_out = tb.hopping(np.array([r1 + eps]), MD)
    assert v_in[0] == pytest.approx(v_out[0], rel=1e-6)
    assert d_in[0] == pytest.approx(d_out[0], rel=1e-5)
    z = 2.0 * np.exp(-(r1 - 1.5) / 0.5)
    B = tb.tail_coefficients(z, -z / 0.5, z / 0.25, r1, rc)
    x = rc - r1
    assert sum(B[k] * x ** k for k in range(6)) == pytest.approx(0, abs=1e-13)
    assert sum(k * B[k] * x ** (k - 1) for k in range(1, 6)) == pytest.approx(0, abs=1e-12)
    assert sum(k * (k - 1) * B[k] * x ** (k - 2) for k in range(2, 6)) == pytest.approx(0, abs=1e-11)
    assert B[2] == pytest.approx(z / 0.25 / 2)          # t''(R1)/2
    v, _ = tb.hopping(np.array([rc, rc + 0.1]), MD)
    assert not v.any()


def test_radial_derivative_by_finite_differences():
    r = np.linspace(1.0, 3.99, 57)
    for m in (M, MD):
        _, d = tb.hopping(r, m)
        h = 1e-6
        fd = (tb.hopping(r + h, m)[0] - tb.hopping(r - h, m)[0]) / (2 * h)
        np.testing.assert_allclose(d, fd, rtol=1e-6, atol=1e-9)


def test_block_gradient_by_finite_differences():
    rng = np.random.default_rng(3)
    for _ in range(5):
        dv = rng.normal(size=3)
        dv *= rng.uniform(1.2, 3.9) / np.linalg.norm(dv)
        G = tb.sk_block_grad(dv, MD)
        for a in range(3):
            e = np.zeros(3)
            e[a] = 1e-6
            fp = tb.sk_block((dv + e) / np.linalg.norm(dv + e), tb.hopping(np.array([np.linalg.norm(dv + e)]), MD)[0][0])
            fm = tb.sk_block((dv - e) / np.linalg.norm(dv - e), tb.hopping(np.array([np.linalg.norm(dv - e)]), MD)[0][0])
            np.testing.assert_allclose(G[a], (fp - fm) / 2e-6, atol=1e-7)


def test_gamma_and_charge_shift():
    pos = np.array([[0.0, 0, 0], [2.0, 0, 0], [0, 3.0, 0]])
    g = tb.gamma_matrix(pos, M)
    assert g[0, 0] == 4.0
    assert g[0, 1] == pytest.approx(synth.COULOMB_EV_A / 2.0)
    assert g[1, 2] == pytest.approx(synth.COULOMB_EV_A / np.sqrt(13.0))
    n = np.array([0.5, -0.25, 0.1])
    H = tb.hamiltonian(pos, n, M)
    V = g @ n
    np.testing.assert_allclose(np.diag(H) - np.diag(tb.hamiltonian0(pos, M)), np.repeat(V, 4))
