"""Write the oracle's reference values for the full-size GPU parity tests.

Test infrastructure: calls only ``oracle/`` and the seeded inputs of
``synth/``; nothing here touches the GPU library.  The oracle is too slow to
run inside a GPU test at these sizes (about 20 s per density matrix at
N = 4096 and 40 s per product at N = 16384 on eight host cores), so its
results are stored once:

* ``c1_xlbomd_n4096.npz`` — the 1024-atom XL-BOMD workload (8 x 8 x 16
  jittered lattice, seed 1, Maxwell velocities at 300 K seed 101, the MD
  model with its hopping tail and pair repulsion): the self-consistent start
  charges (linear mixing from the +-4 e checkerboard), one Born-Oppenheimer
  evaluation at them (H[n] on sampled entries, q, band energy 2 Tr[D H[n]],
  U, forces), and ten XL-BOMD steps of 0.25 fs from them (General remarks
  subsection; Eq. Verl_n with K = 5): energies per step and the final
  positions, velocities, charges and auxiliary-charge history.
* ``c2_mixed_n8192.npz`` — the FP64 SP2 solve of the 2048-atom 8 x 16 x 16
  lattice (seed 2, static model) that the reduced-precision products are
  measured on: branches, traces and idempotency error per product, the
  diagonal of D, D applied to two seeded Gaussian probe vectors, eight sampled
  32 x 32 blocks of D and its squared Frobenius norm.
* ``c3p_blocksparse_permuted_n16384.npz`` — the same thresholded solve with
  the lattice's 8-atom rows (one 32-orbital block each) in a seeded random
  order (``synth.permuted_groups``): as block-sparse, but with the nonzero
  blocks scattered instead of banded.
* ``c3_blocksparse_n16384.npz`` — the thresholded SP2 solve of the
  elongated 8 x 8 x 64 lattice (seed 3, static model), 32 x 32 blocks with
  Frobenius norm below tau = 1e-5 dropped after X_0 and after every update
  (Linear scaling section; block form of the threshold): the branch of each
  update, traces and idempotency error of each product, the fraction of
  blocks kept after each update, the diagonal of D, D applied to two seeded
  Gaussian probe vectors, and eight sampled 32 x 32 blocks of D.

Usage: python tests/golden/make_oracle_golden.py [c1] [c2] [c3] [c3p]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import sp2 as osp2, tb as otb, xlbomd as oxl  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
C1_FILE = os.path.join(HERE, "c1_xlbomd_n4096.npz")
C2_FILE = os.path.join(HERE, "c2_mixed_n8192.npz")
C3_FILE = os.path.join(HERE, "c3_blocksparse_n16384.npz")
C3P_FILE = os.path.join(HERE, "c3p_blocksparse_permuted_n16384.npz")

C1_STEPS = 10
C3_TAU = 1e-5
h_sample_index, probe_vectors, block_index = synth.h_sample_index, synth.probe_vectors, synth.block_index


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def c1_inputs():
    w = synth.XLBOMD
    m = synth.MD_MODEL
    pos = w.positions()
    vel = synth.maxwell_velocities(w.n_atoms, 300.0, m.mass, seed=synth.XLBOMD_VEL_SEED)
    return w, m, pos, vel


def make_c1():
    w, m, pos, vel = c1_inputs()
    n_occ = w.n_occ
    t0 = time.time()
    q_scf, its = oxl.scf(pos, m, n_occ, beta=1.0, tol=1e-11, n0=synth.checkerboard_charges(w.dims))
    log(f"c1: SCF {its} iterations in {time.time() - t0:.0f} s")
    ev = oxl.evaluate(pos, q_scf, m, n_occ)
    H, D = ev["H"], ev["D"]
    hi, hj = h_sample_index(H.shape[0])
    opts = oxl.XLOptions()
    st = oxl.XLState(pos.copy(), vel.copy(), [q_scf.copy() for _ in range(len(opts.c))], ev["q"], ev["F"],
                     ev["U"])
    out = dict(scf_q=q_scf, scf_iterations=its, h_i=hi, h_j=hj, h_val=H[hi, hj], q0=ev["q"], U0=ev["U"],
               F0=ev["F"], e_band0=2.0 * float(np.sum(D * H)), etot0=oxl.total_energy(st, m))
    del H, D, ev
    st, recs = oxl.run(st, m, n_occ, opts, C1_STEPS)
    log(f"c1: {C1_STEPS} steps done at {time.time() - t0:.0f} s")
    out.update(etot=np.array([r["etot"] for r in recs]), U=np.array([r["U"] for r in recs]),
               max_q_minus_n=np.array([r["max_q_minus_n"] for r in recs]),
               pos=st.pos, vel=st.vel, q=st.q, hist=np.array(st.hist))
    np.savez_compressed(C1_FILE, **out)
    log(f"c1: wrote {C1_FILE}")


def solve_summary(r, N, **extra):
    """Arrays stored for a full-size SP2 solve: its steps and samples of D."""
    D = r.D
    nb = (N + 31) // 32
    bi, bj = block_index(nb)
    blocks = np.stack([D[32 * a:32 * a + 32, 32 * b:32 * b + 32] for a, b in zip(bi, bj)])
    return dict(iterations=r.iterations, status=r.status, branches=np.array(r.branches),
                idem=np.array(r.idem), traces=np.array(r.traces), fill=np.array(r.fill),
                eps=np.array([r.eps_min, r.eps_max]), diag=np.diag(D).copy(), DV=D @ probe_vectors(N),
                block_i=bi, block_j=bj, blocks=blocks, fro2=float(np.sum(D * D)), **extra)


def make_c2():
    w = synth.MIXED
    H = otb.hamiltonian(w.positions(), None, synth.STATIC_MODEL)
    t0 = time.time()
    r = osp2.sp2(H, w.n_occ, tol=1e-10)
    log(f"c2: {r.iterations} products, status {r.status}, in {time.time() - t0:.0f} s")
    del H
    np.savez_compressed(C2_FILE, **solve_summary(r, w.n_orb))
    log(f"c2: wrote {C2_FILE}")


def make_c3():
    w = synth.SPARSE
    H = otb.hamiltonian(w.positions(), None, synth.STATIC_MODEL)
    t0 = time.time()
    r = osp2.sp2(H, w.n_occ, tol=1e-10, tau=C3_TAU, threshold="block")
    log(f"c3: {r.iterations} products, status {r.status}, in {time.time() - t0:.0f} s")
    del H
    np.savez_compressed(C3_FILE, **solve_summary(r, w.n_orb, tau=C3_TAU))
    log(f"c3: wrote {C3_FILE}")


def make_c3p():
    w = synth.SPARSE
    H = otb.hamiltonian(synth.permuted_groups(w.positions(), synth.PERMUTED_SEED), None, synth.STATIC_MODEL)
    t0 = time.time()
    r = osp2.sp2(H, w.n_occ, tol=1e-10, tau=C3_TAU, threshold="block")
    log(f"c3p: {r.iterations} products, status {r.status}, in {time.time() - t0:.0f} s")
    del H
    np.savez_compressed(C3P_FILE, **solve_summary(r, w.n_orb, tau=C3_TAU))
    log(f"c3p: wrote {C3P_FILE}")


if __name__ == "__main__":
    which = sys.argv[1:] or ["c1", "c2", "c3", "c3p"]
    for k in which:
        {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c3p": make_c3p}[k]()
