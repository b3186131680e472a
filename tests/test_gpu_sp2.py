"""GPU parity of the dense SP2 path (through the C-ABI) against the CPU oracle."""
import sys

import numpy as np
import pytest

import synth
from oracle import eig, observables, sp2 as osp2, sp2_fp32 as osp2_32, tb as otb

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_1203_6836_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = p.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def oracle_H(dims, seed, model=synth.STATIC_MODEL):
    pos = synth.lattice_positions(dims, seed=seed)
    return pos, otb.hamiltonian(pos, None, model)


# sizes: one full tile, ragged single tile, several tiles with a ragged tail
CASES = [((4, 4, 4), 0), ((3, 3, 3), 7), ((5, 5, 5), 11), ((6, 6, 5), 12)]


@pytest.mark.parametrize("dims,seed", CASES)
def test_fp64_density_matrix_matches_oracle(ctx, dims, seed):
    import paper_1203_6836_amd as p
    say(f"case fp64 dims={dims} seed={seed}")
    pos, H = oracle_H(dims, seed)
    nocc = 2 * len(pos)
    ref = osp2.sp2(H, nocc, tol=1e-10)
    D, st = ctx.sp2_density_matrix(to_dev(H), nocc, p.options("fp64"))
    D = D.cpu().numpy()
    N = H.shape[0]
    err = np.linalg.norm(D - ref.D) / np.sqrt(N)
    say(f"  iters gpu={st['iterations']} oracle={ref.iterations} err/sqrtN={err:.2e} idem={st['idem_err']:.2e}")
    assert err <= 1e-10
    assert np.max(np.abs(D - ref.D)) < 1e-10
    assert st["status"] == "converged"
    assert abs(st["iterations"] - ref.iterations) <= 1
    assert st["eps_min"] == pytest.approx(ref.eps_min, abs=1e-12)
    assert st["eps_max"] == pytest.approx(ref.eps_max, abs=1e-12)
    assert np.array_equal(D, D.T)
    assert abs(np.trace(D) - nocc) < 1e-10
    if st["iterations"] == ref.iterations:
        assert st["branches"] == ref.branches


def test_fp64_equals_jacobi_projector(ctx):
    import paper_1203_6836_amd as p
    say("case fp64 vs jacobi 4x4x4")
    pos, H = oracle_H((4, 4, 4), 0)
    nocc = 2 * len(pos)
    rho, ev, gap = eig.density_matrix(H, nocc)
    D, st = ctx.sp2_density_matrix(to_dev(H), nocc, p.options("fp64"))
    D = D.cpu().numpy()
    assert np.linalg.norm(D - rho) / np.sqrt(H.shape[0]) < 1e-10
    assert np.linalg.norm(H @ D - D @ H) < 1e-9


def test_deterministic_repeat(ctx):
    import paper_1203_6836_amd as p
    say("case determinism 5x5x5")
    _, H = oracle_H((5, 5, 5), 11)
    Hd = to_dev(H)
    D1, s1 = ctx.sp2_density_matrix(Hd, 250, p.options("fp64"))
    D2, s2 = ctx.sp2_density_matrix(Hd, 250, p.options("fp64"))
    assert bool((D1 == D2).all())
    assert s1["branches"] == s2["branches"]


def test_observables_match_oracle(ctx):
    import paper_1203_6836_amd as p
    say("case mulliken/band energy 4x4x4")
    pos, H = oracle_H((4, 4, 4), 0)
    nocc = 2 * len(pos)
    Hd = to_dev(H)
    D, _ = ctx.sp2_density_matrix(Hd, nocc, p.options("fp64"))
    q = ctx.sp2_mulliken(D, len(pos)).cpu().numpy()
    Dn = D.cpu().numpy()
    np.testing.assert_allclose(q, observables.mulliken(Dn), atol=1e-13)
    ref = osp2.sp2(H, nocc)
    assert np.max(np.abs(q - observables.mulliken(ref.D))) <= 1e-9
    e = ctx.sp2_band_energy(D, Hd)
    assert e == pytest.approx(observables.band_energy(ref.D, H), abs=1e-8)


def test_edge_cases_and_errors(ctx):
    import paper_1203_6836_amd as p
    say("case edge: diagonal, tiny, errors")
    d = np.array([-3.0, 1.0, -2.0, 4.0, 0.0, -1.0, 2.5, -0.5])
    D, st = ctx.sp2_density_matrix(to_dev(np.diag(d)), 4, p.options("fp64"))
    np.testing.assert_allclose(np.diag(D.cpu().numpy()), (d <= -0.5).astype(float), atol=1e-12)
    # N = 1 has no valid n_occ; n_occ out of range -> EINVAL
    st_, _ = ctx.sp2_density_matrix_status(to_dev(np.diag(d)), 0)
    assert st_ == p.SP2_EINVAL
    st_, _ = ctx.sp2_density_matrix_status(to_dev(np.diag(d)), 8)
    assert st_ == p.SP2_EINVAL
    # too few products -> ENOCONV (outputs untouched)
    _, H = oracle_H((3, 3, 3), 7)
    st_, stats = ctx.sp2_density_matrix_status(to_dev(H), 54, p.options("fp64", max_iter=3))
    assert st_ == p.SP2_ENOCONV and stats["iterations"] == 3
    # bad option
    st_, _ = ctx.sp2_density_matrix_status(to_dev(H), 54, p.options("fp64", max_iter=500))
    assert st_ == p.SP2_EINVAL


def test_fp64_n2048_against_oracle(ctx):
    import paper_1203_6836_amd as p
    say("case fp64 8x8x8 (N=2048)")
    pos, H = oracle_H((8, 8, 8), 2)
    nocc = 2 * len(pos)
    ref = osp2.sp2(H, nocc)
    D, st = ctx.sp2_density_matrix(to_dev(H), nocc, p.options("fp64"))
    err = np.linalg.norm(D.cpu().numpy() - ref.D) / np.sqrt(H.shape[0])
    say(f"  iters={st['iterations']} err/sqrtN={err:.2e} ms={st['ms']:.1f}")
    assert err <= 1e-10


@pytest.mark.parametrize("dims,seed", [((8, 8, 16), 1), ((8, 16, 16), 2)])
def test_fp64_tail_split(ctx, dims, seed):
    """FP64 products whose last wave of tiles is split along K (N = 4096: 16
    of 528 tiles into 16 chunks; N = 8192: 32 of 2080) against the same solve
    without the split: same products and branches, D equal to rounding."""
    import torch
    import paper_1203_6836_amd as p
    say(f"case fp64 tail split on/off dims={dims}")
    pos = synth.lattice_positions(dims, seed=seed)
    H = ctx.tb_hamiltonian(synth.STATIC_MODEL, to_dev(pos))
    nocc = 2 * len(pos)
    D0, s0 = ctx.sp2_density_matrix(H, nocc, p.options("fp64", tail_split=0))
    D1, s1 = ctx.sp2_density_matrix(H, nocc, p.options("fp64"))
    d = float(torch.linalg.norm(D1 - D0)) / H.shape[0] ** 0.5
    say(f"  iters {s0['iterations']} / {s1['iterations']}  ms {s0['ms']:.1f} / {s1['ms']:.1f}  "
        f"|dD|/sqrtN {d:.2e}")
    assert s0["iterations"] == s1["iterations"]
    assert s0["branches"] == s1["branches"]
    assert d <= 1e-12
    D2, _ = ctx.sp2_density_matrix(H, nocc, p.options("fp64"))
    assert torch.equal(D1, D2)           # deterministic


def test_fp64_n4096_split_against_oracle(ctx):
    """The split FP64 path (N = 4096) against the oracle's SP2 loop."""
    import paper_1203_6836_amd as p
    say("case fp64 8x8x16 (N=4096, tail split) vs oracle")
    pos, H = oracle_H((8, 8, 16), 1)
    nocc = 2 * len(pos)
    ref = osp2.sp2(H, nocc)
    D, st = ctx.sp2_density_matrix(to_dev(H), nocc, p.options("fp64"))
    err = np.linalg.norm(D.cpu().numpy() - ref.D) / np.sqrt(H.shape[0])
    say(f"  iters gpu={st['iterations']} oracle={ref.iterations} err/sqrtN={err:.2e}")
    assert st["iterations"] == ref.iterations
    assert err <= 1e-10


def test_fp64_full_size_properties(ctx):
    """N = 8192 in the benchmark's configuration: properties that hold at any size."""
    import torch
    import paper_1203_6836_amd as p
    say("case fp64 N=8192 properties")
    w = synth.MIXED
    xyz = to_dev(w.positions())
    H = ctx.tb_hamiltonian(synth.STATIC_MODEL, xyz)
    D, st = ctx.sp2_density_matrix(H, w.n_occ, p.options("fp64"))
    say(f"  iters={st['iterations']} ms={st['ms']:.1f} idem={st['idem_err']:.2e}")
    assert st["status"] == "converged"
    D2 = D @ D
    assert float(torch.linalg.norm(D2 - D)) < 1e-9
    assert abs(float(torch.trace(D)) - w.n_occ) < 1e-9
    assert float(torch.linalg.norm(H @ D - D @ H)) < 1e-8
    # sampled rows of H against the oracle's Slater-Koster construction
    pos = w.positions()
    Href = otb.hamiltonian0(pos[:64], synth.STATIC_MODEL)
    np.testing.assert_allclose(H[:256, :256].cpu().numpy(), Href, atol=1e-14)


def degenerate_cases():
    two_atoms = otb.hamiltonian(np.array([[0.0, 0.0, 0.0], [10.0, 0.0, 0.0]]), None, synth.STATIC_MODEL)
    return [(two_atoms, 3), (np.diag([-1.0, 0.0, 0.0, 1.0]), 2), (3.0 * np.eye(4), 2),
            (np.diag([0.0, 1e-13, 2.0]), 1)]


def test_gap_reported_like_the_oracle(ctx):
    import paper_1203_6836_amd as p
    say("case degenerate Fermi level -> SP2_EGAP (fp64, int8x, fp32)")
    for H, nocc in degenerate_cases():
        assert osp2.sp2(H, nocc).status == "gap"
        assert osp2_32.sp2_fp32(H, nocc).status == "gap"
        for prec in ("fp64", "int8x", "fp32"):
            st, stats = ctx.sp2_density_matrix_status(to_dev(H), nocc, p.options(prec))
            assert st == p.SP2_EGAP and stats["status"] == "gap", (H.shape, prec, st, stats["status"])
    # a short budget on the same degenerate pair is ENOCONV, as in the oracle
    H, nocc = degenerate_cases()[1]
    assert osp2.sp2(H, nocc, max_iter=20).status == "max_iter"
    st, stats = ctx.sp2_density_matrix_status(to_dev(H), nocc, p.options("fp64", max_iter=20))
    assert st == p.SP2_ENOCONV and stats["status"] == "max_iter"


def test_invalid_hamiltonian_rejected(ctx):
    import paper_1203_6836_amd as p
    say("case H not symmetric / not finite -> SP2_EINVAL")
    pos = synth.lattice_positions((3, 3, 2), seed=4)
    H = otb.hamiltonian(pos, None, synth.STATIC_MODEL)
    nocc = len(pos) * 2
    scale = np.abs(H).max()
    ok = H.copy()
    ok[0, 5] += 1e-14 * scale                       # within 1e-12 max|H|: accepted
    asym = H.copy()
    asym[7, 40] += 1e-9 * scale
    nan = H.copy()
    nan[3, 3] = np.nan
    inf = H.copy()
    inf[10, 60] = inf[60, 10] = np.inf
    for prec in ("fp64", "int8x"):
        st, stats = ctx.sp2_density_matrix_status(to_dev(ok), nocc, p.options(prec))
        assert st == p.SP2_OK, prec
        for bad in (asym, nan, inf):
            st, stats = ctx.sp2_density_matrix_status(to_dev(bad), nocc, p.options(prec))
            assert st == p.SP2_EINVAL and stats["status"] == "invalid", (prec, st)
            assert stats["iterations"] == 0
    # ragged N (not a multiple of the 32 x 32 check tile) and a large N
    H5 = otb.hamiltonian(synth.lattice_positions((5, 5, 3), seed=9), None, synth.STATIC_MODEL)   # N = 300
    bad5 = H5.copy()
    bad5[299, 0] += 1e-6
    st, _ = ctx.sp2_density_matrix_status(to_dev(bad5), 150, p.options("fp64"))
    assert st == p.SP2_EINVAL
    st, _ = ctx.sp2_density_matrix_status(to_dev(H5), 150, p.options("fp64"))
    assert st == p.SP2_OK


def test_smallest_system_and_unaligned_trace(ctx):
    """N = 2 with one occupied state (FP64, int8 and FP32 products, one padded
    tile) against the eigenvector projector; the band energy on operands that
    are not 16-byte aligned (the scalar branch) equals the aligned one."""
    import torch
    import paper_1203_6836_amd as p
    say("case N=2, unaligned band energy")
    H = np.array([[-1.0, 0.3], [0.3, 0.5]])
    w, V = np.linalg.eigh(H)
    ref = np.outer(V[:, 0], V[:, 0])
    tol = {"fp64": 1e-12, "int8x": 1e-7, "fp32": 1e-6}
    for prec in ("fp64", "int8x", "fp32"):
        D, st = ctx.sp2_density_matrix(to_dev(H), 1, p.options(prec))
        err = np.abs(D.cpu().numpy() - ref).max()
        say(f"  {prec}: iters {st['iterations']} max err {err:.1e}")
        assert err <= tol[prec]
    pos, H = oracle_H((4, 4, 4), 0)
    Hd = to_dev(H)
    D, _ = ctx.sp2_density_matrix(Hd, 2 * len(pos), p.options("fp64"))
    e0 = ctx.sp2_band_energy(D, Hd)
    n = H.shape[0]
    # copies that start one element into a larger buffer: 8-byte but not 16-byte aligned
    bufD = torch.zeros(n * n + 1, dtype=torch.float64, device="cuda")
    bufH = torch.zeros(n * n + 1, dtype=torch.float64, device="cuda")
    Du = bufD[1:].view(n, n)
    Hu = bufH[1:].view(n, n)
    Du.copy_(D)
    Hu.copy_(Hd)
    assert Du.data_ptr() % 16 == 8
    e1 = ctx.sp2_band_energy(Du, Hu)
    ref_e = 2.0 * float(np.sum(D.cpu().numpy() * H))
    say(f"  band energy aligned {e0:.12f} unaligned {e1:.12f} numpy {ref_e:.12f}")
    assert abs(e0 - ref_e) <= 1e-9 * abs(ref_e)
    assert abs(e1 - ref_e) <= 1e-9 * abs(ref_e)


def test_context_reuse_across_sizes(ctx):
    """One context solving large, small, then medium systems gives bitwise the
    results of a fresh context per system (scratch grows and is reused)."""
    import torch
    import paper_1203_6836_amd as p
    say("case context reuse across sizes")
    systems = [((8, 8, 16), 1), ((3, 3, 3), 7), ((6, 6, 5), 12)]
    Hs = []
    for dims, seed in systems:
        pos = synth.lattice_positions(dims, seed=seed)
        Hs.append((ctx.tb_hamiltonian(synth.STATIC_MODEL, to_dev(pos)), 2 * len(pos)))
    for prec in ("int8x", "fp64"):
        shared = [ctx.sp2_density_matrix(H, n, p.options(prec))[0] for H, n in Hs]
        for (H, n), D in zip(Hs, shared):
            fresh = p.Context(0)
            D1, _ = fresh.sp2_density_matrix(H, n, p.options(prec, tile_group=8))
            D0, _ = ctx.sp2_density_matrix(H, n, p.options(prec, tile_group=8))
            torch.cuda.synchronize()
            fresh.close()
            assert torch.equal(D0, D1), (prec, H.shape)
