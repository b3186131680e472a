"""Calibration of the pair-repulsion amplitude of the MD model (oracle side).

Test infrastructure only (writes nothing; prints the amplitude that the
model parameters in synth/ freeze).  The paper's U(R; n) contains a pair
term E_pair but gives no parameters for this synthetic model.  Reading: the
amplitude A of phi(r) = A exp(-(r - r0) / rho) is the one for which the
self-consistent state of the unjittered 4 x 4 x 4 lattice has zero mean
virial, W = sum_i (R_i - R_c) . F_i = 0.  At fixed charges the forces are
affine in A (E_pair does not enter H), so A = -W(0) / (W(1) - W(0)).

Usage: python -m oracle.calibrate_pair
"""
from __future__ import annotations

import numpy as np

from . import xlbomd


def virial_at(pos, q, m, n_occ, A):
    r = xlbomd.evaluate(pos, q, m.with_(pair_a=A), n_occ)
    return float(np.sum((pos - pos.mean(axis=0)) * r["F"]))


def zero_virial_amplitude(m, dims=(4, 4, 4), spacing=1.5, n0=None):
    """Returns (A, W(0), q*) for model m (its pair_a is ignored) on the
    unjittered lattice of the given spacing; the SCF starts from n0
    (default: the +-4 e checkerboard)."""
    import synth
    pos = synth.lattice_positions(dims, spacing=spacing, jitter=0.0, seed=0)
    n_occ = int(round(m.z_val * len(pos) / 2))
    m0 = m.with_(pair_a=0.0)
    if n0 is None:
        n0 = synth.checkerboard_charges(dims)
    q, _ = xlbomd.scf(pos, m0, n_occ, beta=1.0, tol=1e-11, n0=n0)
    w0 = virial_at(pos, q, m0, n_occ, 0.0)
    w1 = virial_at(pos, q, m0, n_occ, 1.0)
    return -w0 / (w1 - w0), w0, q


if __name__ == "__main__":
    import synth
    A, w0, q = zero_virial_amplitude(synth.MD_MODEL)
    print(f"rho = {synth.MD_MODEL.pair_rho} A: zero-virial amplitude A = {A:.6f} eV "
          f"(W(0) = {w0:.4f} eV, charges {q.min():.4f} .. {q.max():.4f})")
    g = synth.GAPPED_MD_MODEL
    A, w0, q = zero_virial_amplitude(g, spacing=synth.GAPPED_SPACING, n0=np.zeros(64))
    print(f"gapped: rho = {g.pair_rho} A: zero-virial amplitude A = {A:.6f} eV "
          f"(W(0) = {w0:.4f} eV, charges {q.min():.4f} .. {q.max():.4f})")
