"""Block-thresholded SP2 (32 x 32 blocks, Frobenius norm < tau dropped after every update)."""
import sys

import numpy as np
import pytest

import synth
from oracle import sp2 as osp2, tb as otb

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_1203_6836_amd as p
    c = p.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_fp64_threshold_matches_oracle(ctx):
    import paper_1203_6836_amd as p
    say("case fp64 tau=1e-5 on 4x4x16 (N=1024, banded)")
    pos = synth.lattice_positions((4, 4, 16), seed=3)
    H = otb.hamiltonian(pos, None, synth.STATIC_MODEL)
    nocc = 2 * len(pos)
    ref = osp2.sp2(H, nocc, tau=1e-5)
    D, st = ctx.sp2_density_matrix(to_dev(H), nocc, p.options("fp64", tau=1e-5))
    D = D.cpu().numpy()
    err = np.linalg.norm(D - ref.D) / np.sqrt(H.shape[0])
    n_upd = st["iterations"] - 1
    say(f"  iters gpu={st['iterations']} oracle={ref.iterations} err/sqrtN={err:.2e} "
        f"fill {ref.fill[0]:.3f} -> {ref.fill[-1]:.3f}")
    assert st["iterations"] == ref.iterations
    assert err <= 1e-9
    np.testing.assert_allclose(st["fill_hist"][:n_upd], ref.fill[1:1 + n_upd], atol=1e-7)
    assert st["fill_min"] == pytest.approx(min(ref.fill), abs=1e-7)
    # thresholding changes the answer only slightly on this gapless model
    dense = osp2.sp2(H, nocc)
    assert np.linalg.norm(D - dense.D) / np.sqrt(H.shape[0]) < 1e-3


def test_tiny_tau_equals_dense(ctx):
    import paper_1203_6836_amd as p
    say("case tau=1e-300 vs dense")
    pos = synth.lattice_positions((4, 4, 4), seed=0)
    Hd = to_dev(otb.hamiltonian(pos, None, synth.STATIC_MODEL))
    D0, s0 = ctx.sp2_density_matrix(Hd, 128, p.options("fp64"))
    D1, s1 = ctx.sp2_density_matrix(Hd, 128, p.options("fp64", tau=1e-300))
    assert s0["iterations"] == s1["iterations"]
    assert float((D0 - D1).abs().max()) < 1e-12
    assert s1["fill_min"] == 1.0


def test_int8x_threshold_full_size(ctx):
    """The 8 x 8 x 64 elongated lattice (N = 16384): int8 products with tau = 1e-5."""
    import torch
    import paper_1203_6836_amd as p
    say("case int8x tau=1e-5 N=16384")
    w = synth.SPARSE
    H = ctx.tb_hamiltonian(synth.STATIC_MODEL, to_dev(w.positions()))
    Ds, ss = ctx.sp2_density_matrix(H, w.n_occ, p.options("int8x", tau=1e-5))
    Di, si = ctx.sp2_density_matrix(H, w.n_occ, p.options("int8x"))
    D64, s64 = ctx.sp2_density_matrix(H, w.n_occ, p.options("fp64"))
    e_thr = float(torch.linalg.norm(Ds - D64)) / w.n_orb ** 0.5
    e_i8 = float(torch.linalg.norm(Di - D64)) / w.n_orb ** 0.5
    fills = ss["fill_hist"][:ss["iterations"] - 1]
    say(f"  iters thr={ss['iterations']} int8={si['iterations']} fp64={s64['iterations']}")
    say(f"  ms thr={ss['ms']:.0f} int8={si['ms']:.0f} fp64={s64['ms']:.0f}")
    say(f"  err vs dense fp64: thresholded {e_thr:.2e}, unthresholded int8 {e_i8:.2e}")
    say("  fill per update: " + " ".join(f"{f:.3f}" for f in fills))
    assert e_i8 <= 1e-6
    assert e_thr <= 1e-3
    assert fills[0] < 0.5 and ss["fill_min"] < 0.2
    assert abs(float(torch.trace(Ds)) - w.n_occ) < 1e-3
