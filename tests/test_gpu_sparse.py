"""Thresholded SP2: 32 x 32 blocks with Frobenius norm < tau, or elements below
tau (the paper's rule), dropped after every update."""
import sys

import numpy as np
import pytest

import synth
from oracle import sp2 as osp2, tb as otb

pytestmark = pytest.mark.gpu
# ||D - D_ref||_F / sqrt(N) of reduced-precision products against the oracle's
# solve with the same threshold: the mixed-precision tolerance.  An element
# (or block) within the products' rounding of tau can land on the other side
# of it, moving D by about tau there; with the int8 expansion's 1e-10
# relative accuracy this happens to a handful of elements at most (measured
# 1e-10 at N = 2048, 2.5e-7 at N = 8192, 3.5e-7 on the scattered N = 4096 wire).
TOL_D = 1e-6


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


@pytest.mark.parametrize("case,rule", [("8x8x8", 0), ("6x6x5", 0), ("6x6x5", 1), ("sparse", 0)])
def test_dense_switch_is_exact(ctx, case, rule):
    """Thresholded int8 solves give bitwise the same D, products, branches and
    fill per update whether their products switch to the dense tile kernel
    from the first product on (dense_fill 0: rows of X_n encoded whole), at
    the default kept fraction 0.95, or never (dense_fill 2): N = 2048, a
    ragged 720 (padded 768: the padding's digits) under both threshold
    rules, and the 16384-orbital workload, whose products run dense from
    the update where every block is kept."""
    import torch
    import paper_1203_6836_amd as p
    if case == "sparse":
        w = synth.SPARSE
        pos, nocc = w.positions(), w.n_occ
    else:
        pos = synth.lattice_positions(tuple(int(x) for x in case.split("x")), seed=5)
        nocc = 2 * len(pos)
    H = ctx.tb_hamiltonian(synth.STATIC_MODEL, to_dev(pos))
    say(f"case dense switch {case} N={H.shape[0]} rule={rule}")
    res = {}
    for f in (2.0, 0.95, 0.0):
        o = p.options("int8x", tau=1e-5, threshold=rule, dense_fill=f)
        D, st = ctx.sp2_density_matrix(H, nocc, o)
        res[f] = (D, st)
        fills = st["fill_hist"][:st["iterations"] - 1]
        say(f"  dense_fill {f}: {st['iterations']} products, {st['ms']:.1f} ms, fill max {max(fills):.3f}")
    D2, s2 = res[2.0]
    for f in (0.95, 0.0):
        D, st = res[f]
        assert st["iterations"] == s2["iterations"]
        assert st["branches"] == s2["branches"]
        assert st["fill_hist"] == s2["fill_hist"]
        assert torch.equal(D, D2)


def test_dense_fill_is_validated(ctx):
    import paper_1203_6836_amd as p
    H = to_dev(np.diag(np.arange(8.0)))
    with pytest.raises(p.Sp2Error):
        ctx.sp2_density_matrix(H, 4, p.options("int8x", tau=1e-5, dense_fill=-0.5))


def test_threshold_rule_is_validated(ctx):
    import paper_1203_6836_amd as p
    H = to_dev(np.diag(np.arange(8.0)))
    st, _ = ctx.sp2_density_matrix_status(H, 4, p.options("fp64", tau=1e-5, threshold=2))
    assert st == p.SP2_EINVAL


@pytest.mark.parametrize("rule,layers", [(0, 32), (1, 32), (1, 33)])
def test_fp64_threshold_gapped_wire_matches_oracle(ctx, rule, layers):
    """Gapped 4 x 4 x 32 wire (N = 2048), and a ragged 4 x 4 x 33 one
    (N = 2112): FP64 products, against the oracle step by step (iterations,
    fill after every update, D)."""
    import paper_1203_6836_amd as p
    name = ("block", "element")[rule]
    w = synth.gapped_workload(layers)
    say(f"case fp64 tau=1e-5 {name} rule, gapped wire N={w.n_orb}")
    H = otb.hamiltonian0(w.positions(), synth.GAPPED_MODEL)
    ref = osp2.sp2(H, w.n_occ, tau=1e-5, threshold=name)
    D, st = ctx.sp2_density_matrix(to_dev(H), w.n_occ, p.options("fp64", tau=1e-5, threshold=rule))
    D = D.cpu().numpy()
    err = np.linalg.norm(D - ref.D) / np.sqrt(H.shape[0])
    n_upd = st["iterations"] - 1
    say(f"  iters gpu={st['iterations']} oracle={ref.iterations} status {st['status']} ({ref.status}) "
        f"err/sqrtN={err:.2e} fill {ref.fill[0]:.3f} -> {ref.fill[-1]:.3f}")
    assert st["iterations"] == ref.iterations
    assert st["status"] == ref.status
    assert err <= 1e-9
    np.testing.assert_allclose(st["fill_hist"][:n_upd], ref.fill[1:1 + n_upd], atol=1e-7)
    assert st["fill_min"] == pytest.approx(min(ref.fill), abs=1e-7)
    if rule == 1:
        # every surviving element is at least tau in magnitude, the rest are zero
        nz = D[D != 0.0]
        assert np.abs(nz).min() >= 1e-5 or nz.size == 0


@pytest.mark.parametrize("layers", [32, 33, 1])
def test_int8x_elementwise_gapped_wire_vs_oracle(ctx, layers):
    """int8 products with the elementwise rule on the gapped wire (N = 2048; a
    ragged N = 2112 whose last tiles are mostly padding; a one-tile N = 64):
    within the mixed-precision tolerance of the oracle's thresholded solve
    (the threshold itself moves D 200 times further)."""
    import paper_1203_6836_amd as p
    w = synth.gapped_workload(layers)
    say(f"case int8x tau=1e-5 element rule, gapped wire N={w.n_orb}")
    H = otb.hamiltonian0(w.positions(), synth.GAPPED_MODEL)
    ref = osp2.sp2(H, w.n_occ, tau=1e-5, threshold="element")
    dense = osp2.sp2(H, w.n_occ)
    D, st = ctx.sp2_density_matrix(to_dev(H), w.n_occ, p.options("int8x", tau=1e-5, threshold=1))
    D = D.cpu().numpy()
    rn = np.sqrt(H.shape[0])
    err = np.linalg.norm(D - ref.D) / rn
    err_thr = np.linalg.norm(ref.D - dense.D) / rn
    say(f"  iters gpu={st['iterations']} oracle={ref.iterations}; err vs oracle {err:.2e}, "
        f"oracle thresholded vs dense {err_thr:.2e}, trace {np.trace(D) - w.n_occ:+.1e}")
    assert abs(st["iterations"] - ref.iterations) <= 1
    assert err <= TOL_D
    assert abs(np.trace(D) - w.n_occ) < 1e-4


def test_int8x_threshold_after_fp64_head_vs_oracle(ctx):
    """Thresholded int8 solve whose first 3 products are FP64 (fp64_head = 3):
    the int8 products then run on the full grid of tiles, diagonal by
    diagonal, without zero-tile flags, from the band-limited encode.  Both
    rules against the oracle on the gapped 4 x 4 x 32 wire (N = 2048), to the
    mixed-precision tolerance like the list-driven path."""
    import paper_1203_6836_amd as p
    w = synth.gapped_workload(32)
    H = otb.hamiltonian0(w.positions(), synth.GAPPED_MODEL)
    dense = osp2.sp2(H, w.n_occ)
    rn = np.sqrt(H.shape[0])
    for rule, name in ((0, "block"), (1, "element")):
        say(f"case int8x fp64_head=3 tau=1e-5 {name} rule, gapped wire N=2048")
        ref = osp2.sp2(H, w.n_occ, tau=1e-5, threshold=name)
        D, st = ctx.sp2_density_matrix(to_dev(H), w.n_occ,
                                       p.options("int8x", tau=1e-5, threshold=rule, fp64_head=3))
        D = D.cpu().numpy()
        err = np.linalg.norm(D - ref.D) / rn
        err_thr = np.linalg.norm(ref.D - dense.D) / rn
        say(f"  iters gpu={st['iterations']} ({st['fp64_products']} FP64) oracle={ref.iterations}; "
            f"err vs oracle {err:.2e}, threshold's own {err_thr:.2e}")
        assert st["fp64_products"] == 3
        assert abs(st["iterations"] - ref.iterations) <= 1
        assert err <= TOL_D
        assert abs(np.trace(D) - w.n_occ) < 1e-4


def test_gapped_wire_full_size_against_oracle(ctx):
    """The smallest size of the benchmark's thresholded-scaling leg (gapped
    wire, N = 8192, elementwise tau = 1e-5) against the oracle's thresholded
    SP2: FP64 products step by step (iterations, fill after every update, D),
    and int8 products (five planes; four planes with five levels as
    benchmarked) within the mixed-precision tolerance (the threshold itself
    moves D by 2.2e-4)."""
    import time
    import paper_1203_6836_amd as p
    say("case gapped wire N=8192 elementwise tau=1e-5 vs oracle (full size)")
    w = synth.gapped_workload(128)
    t0 = time.perf_counter()
    H = otb.hamiltonian0(w.positions(), synth.GAPPED_MODEL)
    ref = osp2.sp2(H, w.n_occ, tau=1e-5, threshold="element")
    say(f"  oracle: {ref.iterations} products in {time.perf_counter() - t0:.0f} s, status {ref.status}, "
        f"fill {ref.fill[0]:.4f} -> {max(ref.fill):.4f}")
    Hd = to_dev(H)
    D, st = ctx.sp2_density_matrix(Hd, w.n_occ, p.options("fp64", tau=1e-5, threshold=1))
    D = D.cpu().numpy()
    rn = np.sqrt(w.n_orb)
    err = np.linalg.norm(D - ref.D) / rn
    n_upd = st["iterations"] - 1
    say(f"  fp64: iters {st['iterations']} err/sqrtN {err:.2e}")
    assert st["iterations"] == ref.iterations and st["status"] == ref.status
    assert err <= 1e-9
    np.testing.assert_allclose(st["fill_hist"][:n_upd], ref.fill[1:1 + n_upd], atol=1e-7)
    for recipe in ({}, {"slices": 4, "levels": 5}):
        D8, s8 = ctx.sp2_density_matrix(Hd, w.n_occ, p.options("int8x", tau=1e-5, threshold=1, **recipe))
        D8 = D8.cpu().numpy()
        err8 = np.linalg.norm(D8 - ref.D) / rn
        say(f"  int8 {recipe}: iters {s8['iterations']} err/sqrtN {err8:.2e}, trace {np.trace(D8) - w.n_occ:+.1e}")
        assert abs(s8["iterations"] - ref.iterations) <= 1
        assert err8 <= TOL_D


def test_gapped_wire_thresholded_scaling(ctx):
    """Gapped wires of N = 8192, 16384 and 32768 orbitals: int8 products, the
    elementwise rule at tau = 1e-5.  The kept fraction falls as 1/N and the
    thresholded solve beats the dense one by a growing factor."""
    import torch
    import paper_1203_6836_amd as p
    rows = []
    for L in (128, 256, 512):
        w = synth.gapped_workload(L)
        say(f"case gapped wire N={w.n_orb} int8x tau=1e-5 element")
        H = ctx.tb_hamiltonian(synth.GAPPED_MODEL, to_dev(w.positions()))
        opt = p.options("int8x", tau=1e-5, threshold=1)
        ctx.sp2_density_matrix(H, w.n_occ, opt)            # warm (allocation)
        D, st = ctx.sp2_density_matrix(H, w.n_occ, opt)
        tr = float(torch.trace(D)) - w.n_occ
        dense_ms = None
        if w.n_orb <= 16384:
            Dd, sd = ctx.sp2_density_matrix(H, w.n_occ, p.options("int8x"))
            dense_ms = sd["ms"]
            e = float(torch.linalg.norm(D - Dd)) / w.n_orb ** 0.5
            say(f"  dense int8 {dense_ms:.0f} ms ({sd['iterations']} products); err vs dense {e:.2e}")
            assert e < 1e-3
            del Dd
        say(f"  thresholded {st['ms']:.1f} ms ({st['iterations']} products), fill min {st['fill_min']:.4f} "
            f"max {st['fill_max']:.4f}, trace {tr:+.1e}")
        rows.append((w.n_orb, st["ms"], st["fill_max"], dense_ms, st["iterations"]))
        assert st["status"] in ("converged", "stalled")
        assert abs(tr) < 1e-3
        del D, H
        torch.cuda.empty_cache()
    # kept fraction ~ 1/N: doubling N halves it (to within 20 %)
    for r0, r1 in zip(rows, rows[1:]):
        assert r1[2] < 0.6 * r0[2]
    # measured 48x at N = 16384 (dense products cost 8x per doubling of N,
    # the thresholded solve about 2.5x per product, dense H and D passes
    # included)
    assert rows[1][3] > 20.0 * rows[1][1]
    per_product = [r[1] / r[4] for r in rows]
    assert per_product[2] < 4.0 * per_product[1]


def test_block_mask_on_a_scattered_wire_against_oracle(ctx):
    """The gapped 4 x 4 x 64 wire (N = 4096) with its 8-atom groups (one
    32-orbital block row each) in a seeded random order: as block-sparse as
    the banded wire, but each 128-row panel's nonzero blocks are scattered
    over the whole range, so only the 32 x 32 block masks (not a column
    range) keep the products sparse.  FP64 products against the oracle step
    by step (products, fill after every update, D); int8 products within the
    mixed-precision tolerance.  The masks are kept per 128-row panel (the
    product tile): a panel of four scattered groups has about three quarters
    of its 32-column blocks set, so the scattered solve still costs a few
    times the banded one, but less than the dense one (measured 7.3 ms
    against 2.2 ms banded and 10.7 ms dense; 10.5 ms with column ranges
    alone)."""
    import paper_1203_6836_amd as p
    w = synth.gapped_workload(64)
    pos_band = w.positions()
    pos = synth.permuted_groups(pos_band, synth.PERMUTED_SEED)
    say(f"case block mask: scattered gapped wire N={w.n_orb}, tau=1e-5 element rule")
    H = otb.hamiltonian0(pos, synth.GAPPED_MODEL)
    ref = osp2.sp2(H, w.n_occ, tau=1e-5, threshold="element")
    dense = osp2.sp2(H, w.n_occ)
    Hd = to_dev(H)
    D64, s64 = ctx.sp2_density_matrix(Hd, w.n_occ, p.options("fp64", tau=1e-5, threshold=1))
    rn = np.sqrt(H.shape[0])
    e64 = np.linalg.norm(D64.cpu().numpy() - ref.D) / rn
    n_upd = s64["iterations"] - 1
    say(f"  fp64: products {s64['iterations']} (oracle {ref.iterations}), err {e64:.1e}, "
        f"fill {ref.fill[0]:.3f} -> {max(ref.fill):.3f}")
    assert s64["iterations"] == ref.iterations and s64["status"] == ref.status
    np.testing.assert_allclose(s64["fill_hist"][:n_upd], ref.fill[1:1 + n_upd], atol=1e-7)
    assert e64 <= 1e-9
    opt8 = p.options("int8x", tau=1e-5, threshold=1)
    ctx.sp2_density_matrix(Hd, w.n_occ, opt8)                     # warm
    D8, s8 = ctx.sp2_density_matrix(Hd, w.n_occ, opt8)
    e8 = np.linalg.norm(D8.cpu().numpy() - ref.D) / rn
    err_thr = np.linalg.norm(ref.D - dense.D) / rn
    Hb = to_dev(otb.hamiltonian0(pos_band, synth.GAPPED_MODEL))
    ctx.sp2_density_matrix(Hb, w.n_occ, opt8)
    _, sb = ctx.sp2_density_matrix(Hb, w.n_occ, opt8)
    _, sd = ctx.sp2_density_matrix(Hd, w.n_occ, p.options("int8x"))
    say(f"  int8: products {s8['iterations']}, err {e8:.1e} (threshold's own {err_thr:.1e}); "
        f"{s8['ms']:.1f} ms scattered vs {sb['ms']:.1f} ms banded vs {sd['ms']:.1f} ms dense")
    assert abs(s8["iterations"] - ref.iterations) <= 1
    assert e8 <= TOL_D
    assert s8["ms"] < 0.85 * sd["ms"]


def test_blocksparse_scattered_n16384_fp64_against_oracle(ctx):
    """The 16384-orbital block-thresholded solve with the lattice's 8-atom
    rows in a seeded random order (nonzero blocks scattered instead of
    banded), FP64 products, against the oracle's stored solve step by step:
    products, branches, fill after every update, D (probe-vector estimate,
    all charges, sampled blocks)."""
    import os
    import torch
    import paper_1203_6836_amd as p
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3p_blocksparse_permuted_n16384.npz")
    with np.load(path, allow_pickle=False) as z:
        g = {k: z[k] for k in z.files}
    w = synth.SPARSE
    say("case block-sparse scattered N=16384 fp64 vs oracle")
    H = ctx.tb_hamiltonian(synth.STATIC_MODEL, to_dev(synth.permuted_groups(w.positions(), synth.PERMUTED_SEED)))
    D, st = ctx.sp2_density_matrix(H, w.n_occ, p.options("fp64", tau=float(g["tau"]), threshold=0))
    n_upd = st["iterations"] - 1
    fill_dev = float(np.max(np.abs(np.array(st["fill_hist"][:n_upd]) - g["fill"][1:1 + n_upd])))
    V = torch.from_numpy(synth.probe_vectors(w.n_orb)).cuda()
    E = (D @ V).cpu().numpy() - g["DV"]
    est = float(np.linalg.norm(E) / np.sqrt(E.shape[1]) / np.sqrt(w.n_orb))
    dd = torch.diagonal(D).cpu().numpy() - g["diag"]
    dq = float(np.max(np.abs(2.0 * dd.reshape(w.n_atoms, -1).sum(axis=1))))
    say(f"  products gpu={st['iterations']} oracle={int(g['iterations'])}; max fill dev {fill_dev:.1e}; "
        f"err/sqrtN ~{est:.1e}, max|dq| {dq:.1e}; fill {g['fill'][0]:.3f} -> {g['fill'][-1]:.3f}")
    assert st["iterations"] == int(g["iterations"]) and st["status"] == str(g["status"])
    assert st["branches"] == [int(b) for b in g["branches"]]
    assert fill_dev <= 1e-7
    assert est <= 1e-9 and dq <= 1e-9
    del D, H
    torch.cuda.empty_cache()
