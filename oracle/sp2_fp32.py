"""Oracle: the SP2 recursion with FP32 products (a precision recipe).

Test infrastructure only.  The paper runs SP2 (Linear scaling section; the
recursion is written out in oracle/sp2.py) in double precision; this module
is the FP32 recipe that the reduced-precision configurations use, written
from the same definition with the arithmetic of each step fixed:

* X_0 = (eps_max I - H) / (eps_max - eps_min) from the FP64 Gershgorin
  bounds, then rounded to FP32;
* P = X_n^2 with FP32 operands and FP32 accumulation (a float32 matrix
  product);
* X_{n+1} = P or 2 X_n - P, formed in FP32 (2 X_n is exact, so the second
  branch rounds once);
* the traces Tr X_n, Tr P and the idempotency error ||P - X_n||_F are FP64
  sums over the FP32 values; the branch rule is the FP64 recursion's;
* stop when ||P - X_n||_F < tol, or when n >= 4, the error has not halved
  over two products (e_n >= e_{n-2} / 2) and e_n < stall: the products have
  reached the FP32 rounding floor (reading: the FP64 rule's r = 1 waits for
  an error that no longer falls at all, which rounding noise at the floor
  can postpone; in the quadratic regime two products shrink the error far
  more than by half, so r = 1/2 stops only at the floor).

Parity of this recipe against a GPU run is to FP32 rounding: the sums of a
float32 product are taken in an order the library chooses, so iterates agree
to a few units of 2^-24 per product, not bitwise.
"""
from __future__ import annotations

import numpy as np

from . import sp2 as _sp2

STALL_RATIO_FP32 = 0.5


def product_fp32(X):
    """X^2 with FP32 operands and FP32 accumulation."""
    X = np.asarray(X, dtype=np.float32)
    return X @ X


def update_fp32(X, P, branch):
    """X_{n+1} in FP32: P (branch 0) or 2 X - P (branch 1)."""
    X = np.asarray(X, dtype=np.float32)
    P = np.asarray(P, dtype=np.float32)
    return P if branch == 0 else np.float32(2.0) * X - P


def sp2_fp32(H, n_occ, tol=1e-10, max_iter=100, stall=1e-2):
    """SP2 density matrix of symmetric H with trace n_occ, FP32 products.

    Returns an SP2Result whose D (the last X_n, as float64) and histories
    follow the FP32 arithmetic above.
    """
    H = np.asarray(H, dtype=np.float64)
    eps_min, eps_max = _sp2.gershgorin(H)
    if not eps_max > eps_min:
        return _sp2.SP2Result(np.zeros_like(H), 0, [], [], [], eps_min, eps_max, False, False, [], "gap")
    X = _sp2.sp2_initial(H, eps_min, eps_max).astype(np.float32)
    branches, idem, traces = [], [], []
    for n in range(max_iter):
        P = product_fp32(X)
        X64, P64 = X.astype(np.float64), P.astype(np.float64)
        t1, t2 = float(np.trace(X64)), float(np.trace(P64))
        e = float(np.linalg.norm(P64 - X64))
        idem.append(e)
        traces.append((t1, t2))
        conv = e < tol
        stalled = n >= 4 and e >= STALL_RATIO_FP32 * idem[n - 2] and e < stall
        if conv or stalled:
            status = "gap" if abs(t1 - n_occ) > 0.5 else ("converged" if conv else "stalled")
            return _sp2.SP2Result(X64, n + 1, branches, idem, traces, eps_min, eps_max,
                                  conv, stalled and not conv, [], status)
        b = _sp2.choose_branch(t1, t2, n_occ)
        branches.append(b)
        X = update_fp32(X, P, b)
    status = "gap" if max_iter >= _sp2.GAP_MIN_ITER and idem[-1] >= _sp2.GAP_IDEM else "max_iter"
    return _sp2.SP2Result(X.astype(np.float64), max_iter, branches, idem, traces, eps_min, eps_max,
                          False, False, [], status)
