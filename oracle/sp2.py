"""Oracle: second-order spectral projection (SP2) purification, FP64.

Test infrastructure only.  The paper constructs the zero-temperature density
matrix by "the recursive second order spectral projection method" and, in its
linear-scaling runs, sets to zero every element below a numerical threshold
tau after each individual projection (Linear scaling section; caption of the
isocyanic-acid energy figure).  It cites the method without printing it, so
the steps below are the standard SP2 recursion written from its definition:

* bounds: Gershgorin discs, eps_min = min_i (H_ii - sum_{j!=i} |H_ij|),
  eps_max = max_i (H_ii + sum_{j!=i} |H_ij|);
* start: X_0 = (eps_max I - H) / (eps_max - eps_min), spectrum in [0, 1],
  occupied states (low energies) near 1;
* iterate: P = X_n^2; X_{n+1} = P (pushes eigenvalues towards 0, lowers the
  trace) or X_{n+1} = 2 X_n - P (pushes towards 1, raises the trace),
  whichever has trace closest to N_occ (reading: ties take P);
* stop after computing P = X_n^2 when ||P - X_n||_F < tol (return X_n), or
  when n >= 4, ||P - X_n||_F >= r ||P_{n-2} - X_{n-2}||_F and
  ||P - X_n||_F < stall (return X_n; the idempotency error has reached its
  floor), or after max_iter iterations (not converged); r = 1 without a
  threshold.

Reading for the thresholded runs (the paper is silent on the stop rule): the
dropped elements perturb every X_n, so the idempotency error settles on a
floor set by tau, not by rounding, and there it keeps shrinking by a tiny
amount per product, so "the error no longer falls" (r = 1) may never hold;
the floor also grows with N (about sqrt of the number of elements near tau),
past 1e-2 on the largest systems.  Once e_n < 0.1 every eigenvalue lies
within d < 0.113 of 0 or 1 (lambda (1 - lambda) <= e_n), where one product
of each branch takes d to at most about 4 d^2 < d / 2: an error that falls by
less than half over two products has left the quadratic regime.  With
tau > 0, r = 1/2 and the bound on e_n is max(stall, 0.1).

The paper's threshold zeroes every element whose magnitude is below tau
(threshold="element").  threshold="block" zeroes each 32 x 32 block whose
Frobenius norm is below tau instead; such a block has every element below tau,
so it drops a subset of what the elementwise rule drops.

Reading for a degenerate Fermi level (the paper is silent): theta(mu0 I - H)
is undefined when the N_occ-th and (N_occ+1)-th eigenvalues coincide (or lie
closer than the products can resolve).  Status "gap" is reported when
* the run stops with an idempotent X_n whose trace is not N_occ
  (|Tr X_n - N_occ| > 1/2: a projector has integer trace, so the occupied
  set could not be chosen), e.g. X_0 already a projector of another rank;
* at least GAP_MIN_ITER products were formed without convergence and
  ||X_n^2 - X_n||_F >= 1/16 (eigenvalues still at least 0.067 from 0 and 1:
  the trace-matching branch rule holds a degenerate cluster at a fraction,
  1/2 for a pair, and the iteration never becomes idempotent);
* eps_max == eps_min (H a multiple of I).
A run stopped earlier by a smaller max_iter is "max_iter" (not converged).

Each branch is a polynomial in X_0, so X_n = p_n(X_0) and the eigenvalues of
X_n are p_n applied to those of X_0 (pinned, with the Jacobi projector, in
tests/test_oracle_sp2.py).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class SP2Result:
    D: np.ndarray
    iterations: int          # number of products X_n^2 formed
    branches: list           # 0: X <- X^2, 1: X <- 2X - X^2, per update
    idem: list               # ||X_n^2 - X_n||_F per product
    traces: list             # (Tr X_n, Tr X_n^2) per product
    eps_min: float
    eps_max: float
    converged: bool
    stalled: bool
    fill: list = dataclasses.field(default_factory=list)
    status: str = ""         # "converged", "stalled", "gap" or "max_iter"

    def __post_init__(self):
        if not self.status:
            self.status = "converged" if self.converged else ("stalled" if self.stalled else "max_iter")


GAP_IDEM = 1.0 / 16.0
GAP_MIN_ITER = 100


def gershgorin(H):
    """Gershgorin bounds (eps_min, eps_max) of symmetric H."""
    d = np.diag(H)
    radius = np.sum(np.abs(H), axis=1) - np.abs(d)
    return float(np.min(d - radius)), float(np.max(d + radius))


def sp2_initial(H, eps_min, eps_max):
    """X_0 = (eps_max I - H) / (eps_max - eps_min)."""
    N = H.shape[0]
    return (eps_max * np.eye(N) - H) / (eps_max - eps_min)


def choose_branch(t1, t2, n_occ):
    """0 (X^2) if its trace is at least as close to n_occ as 2X - X^2's, else 1."""
    return 0 if abs(t2 - n_occ) <= abs(2.0 * t1 - t2 - n_occ) else 1


def _blocks(A, bs):
    """A (N x N) zero-padded to whole bs x bs blocks, viewed as
    [block row, row in block, block column, column in block]."""
    N = A.shape[0]
    nb = (N + bs - 1) // bs
    P = np.zeros((nb * bs, nb * bs), dtype=A.dtype)
    P[:N, :N] = A
    return P.reshape(nb, bs, nb, bs), nb


def block_threshold(X, tau, bs=32):
    """Zero every bs x bs block whose Frobenius norm is below tau.

    Returns (thresholded copy, fraction of blocks kept).  Blocks on the
    ragged edge are the partial blocks of the grid (zero padding adds
    nothing to their norms).
    """
    N = X.shape[0]
    B, nb = _blocks(X, bs)
    keep = np.sqrt(np.sum(B * B, axis=(1, 3))) >= tau          # nb x nb
    mask = np.repeat(np.repeat(keep, bs, axis=0), bs, axis=1)[:N, :N]
    return np.where(mask, X, 0.0), int(keep.sum()) / (nb * nb)


def element_threshold(X, tau, bs=32):
    """Zero every element with |x| < tau (the paper's rule).

    Returns (thresholded copy, fraction of bs x bs blocks that still hold a
    nonzero element), the fill measure of the block form.
    """
    Y = np.where(np.abs(X) < tau, 0.0, X)
    B, nb = _blocks(Y != 0.0, bs)
    return Y, int(B.any(axis=(1, 3)).sum()) / (nb * nb)


STALL_RATIO_THRESHOLDED = 0.5
STALL_GUARD_THRESHOLDED = 0.1


def sp2(H, n_occ, tol=1e-10, max_iter=100, stall=1e-2, tau=0.0, block=32,
        bounds=None, threshold="block"):
    """SP2 density matrix of symmetric H with trace n_occ.

    tau > 0 selects the thresholded variant: after X_0 and after every
    update, blocks of size ``block`` with Frobenius norm below tau are zeroed
    (threshold="block") or elements below tau are zeroed (threshold="element",
    the paper's rule); the stall test then uses r = 1/2 and the bound
    max(stall, 0.1).
    """
    if threshold not in ("block", "element"):
        raise ValueError(threshold)
    thr = block_threshold if threshold == "block" else element_threshold
    ratio = STALL_RATIO_THRESHOLDED if tau > 0.0 else 1.0
    if tau > 0.0:
        stall = max(stall, STALL_GUARD_THRESHOLDED)
    H = np.asarray(H, dtype=np.float64)
    eps_min, eps_max = gershgorin(H) if bounds is None else bounds
    if not eps_max > eps_min:
        return SP2Result(np.zeros_like(H), 0, [], [], [], eps_min, eps_max, False, False, [], "gap")
    X = sp2_initial(H, eps_min, eps_max)
    fill = []
    if tau > 0.0:
        X, f = thr(X, tau, block)
        fill.append(f)
    branches, idem, traces = [], [], []
    for n in range(max_iter):
        P = X @ X
        t1, t2 = float(np.trace(X)), float(np.trace(P))
        e = float(np.linalg.norm(P - X))
        idem.append(e)
        traces.append((t1, t2))
        conv = e < tol
        stalled = n >= 4 and e >= ratio * idem[n - 2] and e < stall
        if conv or stalled:
            status = "gap" if abs(t1 - n_occ) > 0.5 else ("converged" if conv else "stalled")
            return SP2Result(X, n + 1, branches, idem, traces, eps_min, eps_max,
                             conv, stalled and not conv, fill, status)
        b = choose_branch(t1, t2, n_occ)
        branches.append(b)
        X = P if b == 0 else 2.0 * X - P
        if tau > 0.0:
            X, f = thr(X, tau, block)
            fill.append(f)
    status = "gap" if max_iter >= GAP_MIN_ITER and idem[-1] >= GAP_IDEM else "max_iter"
    return SP2Result(X, max_iter, branches, idem, traces, eps_min, eps_max,
                     False, False, fill, status)


def scalar_sp2(x0, branches):
    """Apply a branch sequence to scalars: p_n(x) of the spectral mapping."""
    x = np.array(x0, dtype=np.float64)
    for b in branches:
        x = x * x if b == 0 else 2.0 * x - x * x
    return x
