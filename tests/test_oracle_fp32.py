"""Pins of the FP32 SP2 recipe: each product within the FP32 rounding bound of
the exact product of its operands, the update rounded once, the whole
recursion at FP32 distance from the FP64 projector, exact on a diagonal H."""
import numpy as np
import pytest

import synth
from oracle import eig, sp2, sp2_fp32, tb

U32 = 2.0 ** -24          # unit roundoff of FP32


@pytest.fixture(scope="module")
def small():
    w = synth.SMALL
    H = tb.hamiltonian(w.positions(), None, synth.STATIC_MODEL)
    return w, H


def test_product_is_fp32_within_the_rounding_bound(small):
    """|fl(X X) - X X| <= gamma_K (|X| |X|) elementwise (K terms, FP32
    accumulation), and the sums are not the correctly rounded exact ones, as
    a product formed in FP64 and rounded once would be."""
    _, H = small
    lo, hi = sp2.gershgorin(H)
    X = sp2.sp2_initial(H, lo, hi).astype(np.float32)
    P = sp2_fp32.product_fp32(X)
    assert P.dtype == np.float32
    X64 = X.astype(np.float64)
    exact = X64 @ X64                     # FP64: exact to ~1e-16 relative for FP32 operands
    K = X.shape[0]
    gamma = K * U32 / (1.0 - K * U32)
    assert np.all(np.abs(P - exact) <= gamma * (np.abs(X64) @ np.abs(X64)) + 1e-30)
    assert np.count_nonzero(P != exact.astype(np.float32)) > 0.01 * P.size


def test_update_rounds_once():
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, (64, 64)).astype(np.float32)
    P = rng.uniform(-1, 1, (64, 64)).astype(np.float32)
    np.testing.assert_array_equal(sp2_fp32.update_fp32(X, P, 0), P)
    two_x_minus_p = (2.0 * X.astype(np.float64) - P.astype(np.float64)).astype(np.float32)
    np.testing.assert_array_equal(sp2_fp32.update_fp32(X, P, 1), two_x_minus_p)


def test_recipe_tracks_the_fp64_recursion(small):
    """Same branches as the FP64 recursion until the last few products, stops
    at the FP32 floor, and lands at FP32 distance from the FP64 projector:
    far above the FP64 floor, far below the error of the BF16 products."""
    w, H = small
    r64 = sp2.sp2(H, w.n_occ)
    r32 = sp2_fp32.sp2_fp32(H, w.n_occ)
    assert r32.status == "stalled" and r64.status == "converged"
    assert abs(r32.iterations - r64.iterations) <= 3
    n = min(len(r32.branches), len(r64.branches)) - 6
    assert r32.branches[:n] == r64.branches[:n]
    err = np.linalg.norm(r32.D - r64.D) / np.sqrt(H.shape[0])
    assert 1e-7 < err < 5e-5
    assert abs(np.trace(r32.D) - w.n_occ) < 1e-4
    assert 1e-8 < r32.idem[-1] < 1e-3
    # in the quadratic regime, above the floor, two products shrink the
    # error by far more than half (the stall rule's r = 1/2 stops only there)
    quad = [k for k in range(4, len(r32.idem)) if 1e-3 < r32.idem[k - 2] < 0.1]
    assert len(quad) >= 3
    for k in quad:
        assert r32.idem[k] < 0.5 * r32.idem[k - 2]


def test_recipe_is_the_projector_on_a_diagonal_h():
    """Diagonal H with distinct levels: every X_n is diagonal, X_0's entries
    run to exactly 0 or 1 in FP32, and D is the projector on the n_occ lowest."""
    e = np.linspace(-3.0, 2.5, 24)
    H = np.diag(e[::-1])
    ref, _, _ = eig.density_matrix(H, 10)
    r = sp2_fp32.sp2_fp32(H, 10)
    assert r.status in ("converged", "stalled")
    assert np.count_nonzero(r.D - np.diag(np.diag(r.D))) == 0
    assert np.abs(r.D - ref).max() < 1e-6
